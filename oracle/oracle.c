/*
 * FP64 CPU ORACLE for per-node meta-meshing and arc-subdivision triangulation
 * of strut lattices (Zou & Gao, "Warp-centric GPU meta-meshing and fast
 * triangulation of billion-scale lattice structures").
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  The product library never links,
 * calls or includes it, and it shares no code, header or table with the GPU
 * path.  It is written for obviousness, not speed: plain loops in double
 * precision, one node at a time, threads over node ranges.
 *
 * Model (Sec. 4.1, Sec. 4.3.1): every strut is the round cone tangent to the
 * nodal spheres of its two end nodes.  Around a node c of radius rho with
 * incident struts m = 1..v (far node c_m, radius rho_m, L_m = |c_m - c|,
 * e_m = (c_m - c)/L_m, sigma_m = (rho - rho_m)/L_m, kappa_m = sqrt(1-sigma_m^2))
 * write, for a point w = x - c,
 *      S(w)   = |w|^2 - rho^2
 *      P_m(w) = g_m . w - h_m,   g_m = e_m / kappa_m,  h_m = rho sigma_m / kappa_m
 *      P_0(w) = 0.
 * Cone m is S = P_m^2 (P_m is arc length along a generator, measured from the
 * tangency circle), and the local boundary of the union is S = M^2 with
 * M = max(0, P_1..P_v).  Two cones meet where P_p = P_q: the auxiliary plane of
 * Sec. 4.3.1.  Label 0 (the sphere) meets cone q on its tangency circle.
 *
 * Per node the oracle follows the paper's steps in order:
 *   1. conics: the Eq. 7 ellipse of strut p cut by the auxiliary plane
 *      P_p = P_q (and the tangency circle for the pair (0, q));
 *   2. trimming: Eq. 8/9 keeps, on conic (p,q), the parameter set where
 *      P_p >= P_r for every other label r; the kept runs are the arcs;
 *   3. vertices: arc ends are triple ties P_p = P_q = P_r on S = P_p^2, solved
 *      directly and named (p<q<r, root rank along the tie line);
 *   4. arc loops per strut end (Sec. 4.3.1, last paragraph), hole contours
 *      from the circular arcs that border no other strut (Sec. 5);
 *   5. Eq. 11 segment counts, Eq. 12 sub-parameters, Eq. 13 hole centres,
 *      strut bands "connecting these vertices" (Sec. 5) by a phi-merge zipper,
 *      hole fans.
 * Readings where the paper is silent or garbled (alpha as arcsin, per-node
 * radii, several arcs per seam, N = segments capped at k, uniform-t
 * subdivision, zipper apex rule, orientation) are listed in the design notes.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXV 254
#define TWO_PI 6.283185307179586476925286766559

/* which test produced a node's smallest margin */
#define MK_ELLIPSE 1  /* seam conic close to a parabola */
#define MK_CONIC 2    /* |F| at an extremum of F = min_r f_r on a conic */
#define MK_FRAME 3    /* strut-frame axis choice (full circles only) */
#define MK_ROOTS 4    /* two roots of a triple tie close together */
#define MK_GAP 5      /* runner-up strut close at a vertex (near 4-way tie) */
#define MK_FLOOR 6    /* k dt / 2 pi close to an integer (Eq. 11 floor) */
#define MK_HOLE 7     /* hole barycentre close to the node centre */
#define MK_STEP 8     /* small phi step along a loop */
#define MK_N 9       /* margin kinds 1..8 */
/* lowers the node's margin and the margin of its kind */
#define LOWER(val, kind)                                                      \
    do {                                                                      \
        double v_ = (val);                                                    \
        if (v_ < margin) { margin = v_; mkind = (kind); }                     \
        if (v_ < kmin[(kind)]) kmin[(kind)] = v_;                             \
    } while (0)

/* node status bits */
#define ST_INVALID_STRUT 1u
#define ST_NON_ELLIPTIC 2u
#define ST_LOOP 4u
#define ST_TOPOLOGY 8u
#define ST_ISOLATED 16u
#define ST_VALENCE 32u
#define ST_DUPLICATE 64u

typedef struct {
    double x, y, z;
} V3;

static inline V3 mk(double x, double y, double z) { V3 r = {x, y, z}; return r; }
static inline V3 add(V3 a, V3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline V3 sub(V3 a, V3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline V3 scl(V3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline V3 cross(V3 a, V3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline double nrm(V3 a) { return sqrt(dot(a, a)); }
static inline V3 unit(V3 a) { return scl(a, 1.0 / nrm(a)); }

static uint32_t vname(int a, int b, int c, int root)
{
    return ((uint32_t)a << 24) | ((uint32_t)b << 16) | ((uint32_t)c << 8) | (uint32_t)root;
}

/* ------------------------------------------------------------------ */
/* per-node data                                                        */

typedef struct {
    int p, q;
    V3 o, a, b;   /* x(t) = c + o + a sin t + b cos t (Eq. 1), o local */
    double t1, t2; /* kept range, t2 > t1 */
    int full;
    int rs, re;   /* constraint labels ending the arc at t1 / t2 */
    uint32_t ns, ne_; /* vertex names at t1 / t2 */
    int vs, ve;   /* local vertex indices at t1 / t2 */
    int nseg;
    int contour;  /* hole contour id for circular arcs */
    int mbase;    /* local mesh index of the first interior point */
} Arc;

typedef struct {
    uint32_t name;
    V3 w;
    double sep, gap; /* root separation and runner-up gap (units of rho) */
} Vert;

typedef struct {
    int status;
    double margin;     /* min normalised margin (topology + geometry) */
    int margin_kind;   /* which test set the margin (MK_* codes) */
    double kmargin[MK_N]; /* smallest margin of each kind (index MK_*) */
    int v;
    int nv, ne, nc;
    Vert *verts;       /* sorted by name */
    Arc *arcs;         /* canonical order (p, q, min endpoint name) */
    /* loops: label m (1..v) -> arcs loop_arc[loop_off[m-1] .. loop_off[m]) */
    int *loop_off, *loop_arc, *loop_dir;
    /* k dependent */
    int nmesh, nfan;
    double *mesh_w;    /* 3*nmesh local positions */
    int *fan;          /* 3*nfan local mesh indices */
    int *lv_off;       /* per label: loop vertex sequence offsets (v+1) */
    int *lv_idx;       /* local mesh index */
    double *lv_phi;
    uint8_t *lv_whole; /* the sample lies on a whole tangency circle */
    double *cont_b;    /* hole centre (local) per contour, 3*nc */
} NodeRes;

typedef struct {
    /* inputs */
    int64_t N, S;
    const double *X, *R;   /* X: 3N, R: N */
    const int32_t *sa, *sb;
    int k;
    /* adjacency */
    int64_t *off;          /* N+1 */
    int32_t *adj;          /* 2S strut ids, sorted per node */
    /* results */
    NodeRes *nodes;
    /* global mesh */
    int64_t *mesh_off;     /* N+1 */
    int64_t *band_off;     /* S+1 */
    int64_t *fan_off;      /* N+1 */
    int64_t n_mesh, n_band, n_fan;
    double *mesh;          /* 3 * n_mesh absolute */
    int64_t *tri;          /* 3 * (n_band + n_fan) */
    double *strut_margin;  /* S */
    int *strut_status;     /* S: 0 ok, 1 skipped because an end node is flagged */
    /* threading */
    int64_t next;
    int nthreads;
} Ctx;

/* Everything the node computation needs about one incident strut. */
typedef struct {
    int v;
    V3 c;
    double rho;
    int far[ORC_MAXV + 1], sid[ORC_MAXV + 1], lower[ORC_MAXV + 1];
    V3 e[ORC_MAXV + 1], g[ORC_MAXV + 1], es[ORC_MAXV + 1], rh[ORC_MAXV + 1], qh[ORC_MAXV + 1];
    double h[ORC_MAXV + 1], sig[ORC_MAXV + 1], kap[ORC_MAXV + 1], len[ORC_MAXV + 1];
    double frame_gap[ORC_MAXV + 1];
} Local;

/* ------------------------------------------------------------------ */
/* Step 1: conics                                                       */

/* Canonical frame of a strut (used for phi and for circles): e_s points from
 * the lower node id to the higher one; r = unit(e_s x axis_j) where axis j is
 * the coordinate axis with the smallest |e_s,j| (lowest index on ties);
 * q = e_s x r.  Returns the gap to the next-smallest |e_s,j|. */
static double strut_frame(V3 es, V3 *r, V3 *q)
{
    double ax[3] = {fabs(es.x), fabs(es.y), fabs(es.z)};
    int j = 0;
    for (int i = 1; i < 3; ++i)
        if (ax[i] < ax[j]) j = i;
    double gap = 1e300;
    for (int i = 0; i < 3; ++i)
        if (i != j && ax[i] - ax[j] < gap) gap = ax[i] - ax[j];
    V3 axis = mk(j == 0, j == 1, j == 2);
    *r = unit(cross(es, axis));
    *q = cross(es, *r);
    return gap;
}

/* Eq. 7: ellipse cut from strut p's cone by the auxiliary plane P_p = P_q.
 * d is the unit direction from the far end towards the node, alpha the cone
 * half-angle arcsin((r1 - r0)/L) (arccos as printed gives pi/2 for a cylinder
 * instead of 0), F1/F2 the tangency-circle points in the plane through the axis
 * and the plane normal, E1/E2 where the generators through F1/F2 hit the plane
 * (the major-axis ends).  Returns -1 if the section is not an ellipse.
 * Canonical signs: a . g_p > 0 and b = lambda (a x n) with n = unit(g_p - g_q). */
static int conic_ellipse(const Local *L, int p, int q, V3 *o, V3 *a, V3 *b, double *ell_margin)
{
    V3 n = sub(L->g[p], L->g[q]);
    double nn = nrm(n);
    V3 nh = scl(n, 1.0 / nn);
    V3 ppl = scl(nh, (L->h[p] - L->h[q]) / nn);
    double en = dot(L->e[p], nh);
    *ell_margin = fabs(en) - fabs(L->sig[p]);
    if (*ell_margin <= 0.0) return -1;
    V3 d = scl(L->e[p], -1.0);
    double r0 = L->rho;
    double alpha = asin(-L->sig[p]); /* sin(alpha) = (r1 - r0)/L */
    V3 dp = cross(d, nh);
    if (nrm(dp) < 1e-14) { /* plane normal along the axis: any perpendicular */
        V3 t = fabs(d.x) < 0.9 ? mk(1, 0, 0) : mk(0, 1, 0);
        dp = cross(d, t);
    }
    dp = unit(dp);
    V3 dxd = cross(dp, d); /* Rot(dp, th) d = d cos th + (dp x d) sin th */
#define ROT(th) add(scl(d, cos(th)), scl(dxd, sin(th)))
    V3 F1 = scl(ROT(alpha - M_PI / 2), r0);
    V3 F2 = scl(ROT(M_PI / 2 - alpha), r0);
    V3 G1 = ROT(alpha);
    V3 G2 = ROT(-alpha);
#undef ROT
    V3 E1 = add(F1, scl(G1, dot(nh, sub(ppl, F1)) / dot(nh, G1)));
    V3 E2 = add(F2, scl(G2, dot(nh, sub(ppl, F2)) / dot(nh, G2)));
    *o = scl(add(E1, E2), 0.5);
    *a = scl(sub(E1, E2), 0.5);
    double ad = dot(*a, d), ca = cos(alpha), aa = nrm(*a);
    double lam2 = 1.0 - (ad * ad) / (ca * ca * aa * aa);
    double lam = lam2 > 0 ? sqrt(lam2) : 0.0;
    if (dot(*a, L->g[p]) < 0) *a = scl(*a, -1.0);
    *b = scl(cross(*a, nh), lam);
    return 0;
}

/* Tangency circle of strut q (the conic with the sphere, label 0):
 * centre rho sigma_q e_q, radius rho kappa_q, parametrised so t equals the
 * strut-frame angle phi. */
static void conic_circle(const Local *L, int q, V3 *o, V3 *a, V3 *b)
{
    double rad = L->rho * L->kap[q];
    *o = scl(L->e[q], L->rho * L->sig[q]);
    *a = scl(L->qh[q], rad);
    *b = scl(L->rh[q], rad);
}

static inline V3 conic_pt(V3 o, V3 a, V3 b, double t)
{
    return add(o, add(scl(a, sin(t)), scl(b, cos(t))));
}

static inline double Pval(const Local *L, int m, V3 w)
{
    return m == 0 ? 0.0 : dot(L->g[m], w) - L->h[m];
}

/* ------------------------------------------------------------------ */
/* Step 3: triple ties                                                  */

/* The two points where P_a = P_b = P_c on S = P_a^2 (a < b < c), ordered
 * along d = (g_a - g_b) x (g_a - g_c).  Returns the number of real roots. */
static int triple_roots(const Local *L, int a, int b, int c, V3 out[2], double *sep)
{
    V3 ga = a ? L->g[a] : mk(0, 0, 0);
    double ha = a ? L->h[a] : 0.0;
    V3 n1 = sub(ga, L->g[b]), n2 = sub(ga, L->g[c]);
    double d1 = ha - L->h[b], d2 = ha - L->h[c];
    double G11 = dot(n1, n1), G12 = dot(n1, n2), G22 = dot(n2, n2);
    double det = G11 * G22 - G12 * G12;
    if (!(det > 0)) return 0;
    double x1 = (d1 * G22 - d2 * G12) / det, x2 = (d2 * G11 - d1 * G12) / det;
    V3 w0 = add(scl(n1, x1), scl(n2, x2));
    V3 d = cross(n1, n2);
    double gd = dot(ga, d), pw = dot(ga, w0) - ha;
    double qa = dot(d, d) - gd * gd;
    double qb = 2.0 * (dot(w0, d) - gd * pw);
    double qc = dot(w0, w0) - L->rho * L->rho - pw * pw;
    double l1, l2;
    if (fabs(qa) < 1e-300) {
        if (qb == 0) return 0;
        l1 = l2 = -qc / qb;
    } else {
        double disc = qb * qb - 4 * qa * qc;
        if (disc < 0) return 0;
        double sq = sqrt(disc);
        double qq = -0.5 * (qb + (qb >= 0 ? sq : -sq));
        l1 = qq / qa;
        l2 = qq != 0 ? qc / qq : l1;
    }
    if (l1 > l2) { double t = l1; l1 = l2; l2 = t; }
    out[0] = add(w0, scl(d, l1));
    out[1] = add(w0, scl(d, l2));
    *sep = (l2 - l1) * nrm(d) / L->rho;
    return 2;
}

/* ------------------------------------------------------------------ */
/* Step 2: trimming of one conic (Eqs. 8-9)                             */

typedef struct {
    double ang;
    int r;
    int start; /* 1: lower end of a kept interval (P_p - P_r turns >= 0) */
} Brk;

static int brk_cmp(const void *x, const void *y)
{
    const Brk *a = x, *b = y;
    if (a->ang < b->ang) return -1;
    if (a->ang > b->ang) return 1;
    return a->r - b->r;
}

static double wrap2pi(double t)
{
    t = fmod(t, TWO_PI);
    if (t < 0) t += TWO_PI;
    return t;
}

/* coefficients of f_r(t) = P_p(x(t)) - P_r(x(t)) = A sin t + B cos t + C */
static void fcoef(const Local *L, int p, int r, V3 o, V3 a, V3 b, double *A, double *B, double *C)
{
    V3 gp = p ? L->g[p] : mk(0, 0, 0), gr = r ? L->g[r] : mk(0, 0, 0);
    double hp = p ? L->h[p] : 0.0, hr = r ? L->h[r] : 0.0;
    V3 dg = sub(gp, gr);
    *A = dot(dg, a);
    *B = dot(dg, b);
    *C = dot(dg, o) - (hp - hr);
}

typedef struct {
    double t1, t2;
    int rs, re, full;
} RawArc;

/* Kept arcs of conic (p,q).  Returns the number of arcs written to out and
 * lowers *margin to the smallest |F| at a local extremum of
 * F(t) = min_r f_r(t) (tangencies, near-splits, near-4-way ties). */
static int trim_conic(const Local *L, int p, int q, V3 o, V3 a, V3 b, RawArc *out, double *margin)
{
    int v = L->v;
    double A[ORC_MAXV + 1], B[ORC_MAXV + 1], C[ORC_MAXV + 1];
    int nr = 0;
    Brk *br = malloc(sizeof(Brk) * 2 * (v + 1));
    int nb = 0, empty = 0;
    for (int r = 0; r <= v; ++r) {
        if (r == p || r == q) continue;
        fcoef(L, p, r, o, a, b, &A[nr], &B[nr], &C[nr]);
        double R = hypot(A[nr], B[nr]);
        double Cn = C[nr];
        if (Cn >= R) { ++nr; continue; }        /* never active */
        if (Cn <= -R) { empty = 1; ++nr; continue; } /* cuts the whole conic */
        double psi = atan2(A[nr], B[nr]);
        double beta = acos(-Cn / R);
        br[nb].ang = wrap2pi(psi - beta); br[nb].r = r; br[nb].start = 1; ++nb;
        br[nb].ang = wrap2pi(psi + beta); br[nb].r = r; br[nb].start = 0; ++nb;
        ++nr;
    }
    /* margin: |F| at local extrema of F(t) = min_r f_r(t) */
    {
        double Fscale = L->rho;
#define FEVAL(t, Fv)                                                          \
    do {                                                                      \
        double st_ = sin(t), ct_ = cos(t);                                    \
        Fv = 1e300;                                                           \
        for (int j_ = 0; j_ < nr; ++j_) {                                     \
            double f_ = A[j_] * st_ + B[j_] * ct_ + C[j_];                    \
            if (f_ < Fv) Fv = f_;                                             \
        }                                                                     \
    } while (0)
        for (int j = 0; j < nr; ++j) {
            double R = hypot(A[j], B[j]);
            if (R <= 0) continue;
            double psi = atan2(A[j], B[j]);
            for (int s = 0; s < 2; ++s) {
                double t = psi + (s ? M_PI : 0.0);
                double Fv;
                FEVAL(t, Fv);
                double fj = A[j] * sin(t) + B[j] * cos(t) + C[j];
                if (fj <= Fv + 1e-15 * Fscale) {
                    double m = fabs(Fv) / Fscale;
                    if (m < *margin) *margin = m;
                }
            }
        }
        for (int i = 0; i < nr; ++i)
            for (int j = i + 1; j < nr; ++j) {
                double dA = A[i] - A[j], dB = B[i] - B[j], dC = C[i] - C[j];
                double R = hypot(dA, dB);
                if (R <= 0 || fabs(dC) > R) continue;
                double psi = atan2(dA, dB), beta = acos(-dC / R);
                for (int s = 0; s < 2; ++s) {
                    double t = psi + (s ? beta : -beta);
                    double Fv;
                    FEVAL(t, Fv);
                    double fi = A[i] * sin(t) + B[i] * cos(t) + C[i];
                    if (fi <= Fv + 1e-12 * Fscale) {
                        double m = fabs(Fv) / Fscale;
                        if (m < *margin) *margin = m;
                    }
                }
            }
#undef FEVAL
    }
    int na = 0;
    if (empty) { free(br); return 0; }
    if (nb == 0) {
        out[0].t1 = 0.0; out[0].t2 = TWO_PI; out[0].rs = out[0].re = -1; out[0].full = 1;
        free(br);
        return 1;
    }
    qsort(br, nb, sizeof(Brk), brk_cmp);
    for (int i = 0; i < nb; ++i) {
        Brk s = br[i], e = br[(i + 1) % nb];
        double t1 = s.ang, t2 = i + 1 < nb ? e.ang : e.ang + TWO_PI;
        if (!(t2 > t1)) { *margin = 0.0; continue; } /* coincident breakpoints */
        double tm = 0.5 * (t1 + t2);
        int kept = 1;
        for (int j = 0; j < nr; ++j)
            if (A[j] * sin(tm) + B[j] * cos(tm) + C[j] < 0) { kept = 0; break; }
        if (!kept) continue;
        out[na].t1 = t1; out[na].t2 = t2; out[na].rs = s.r; out[na].re = e.r; out[na].full = 0;
        if (!s.start || e.start) *margin = 0.0; /* inconsistent run ends: degenerate */
        ++na;
    }
    free(br);
    return na;
}

/* ------------------------------------------------------------------ */
/* helpers                                                              */

static int find_vert(const Vert *vs, int nv, uint32_t name)
{
    for (int i = 0; i < nv; ++i)
        if (vs[i].name == name) return i;
    return -1;
}

static int vert_cmp(const void *x, const void *y)
{
    const Vert *a = x, *b = y;
    return a->name < b->name ? -1 : (a->name > b->name);
}

static uint32_t arc_key_name(const Arc *a) { return a->ns < a->ne_ ? a->ns : a->ne_; }

static int arc_cmp(const void *x, const void *y)
{
    const Arc *a = x, *b = y;
    if (a->p != b->p) return a->p - b->p;
    if (a->q != b->q) return a->q - b->q;
    uint32_t ka = arc_key_name(a), kb = arc_key_name(b);
    return ka < kb ? -1 : (ka > kb);
}

static double phi_of(const Local *L, int m, V3 w) { return atan2(dot(w, L->qh[m]), dot(w, L->rh[m])); }

static double wrap_pi(double d)
{
    while (d <= -M_PI) d += TWO_PI;
    while (d > M_PI) d -= TWO_PI;
    return d;
}

/* ------------------------------------------------------------------ */
/* one node: arrangement, loops, holes, subdivision                     */

static void node_fail(NodeRes *R, int status)
{
    R->status |= status;
}

static void node_compute(Ctx *X, int64_t n)
{
    NodeRes *R = &X->nodes[n];
    memset(R, 0, sizeof(*R));
    R->margin = 1e300;
    for (int i = 0; i < MK_N; ++i) R->kmargin[i] = 1e300;
    int v = (int)(X->off[n + 1] - X->off[n]);
    R->v = v;
    if (v == 0) { node_fail(R, ST_ISOLATED); return; }
    if (v > ORC_MAXV) { node_fail(R, ST_VALENCE); return; }
    Local *L = calloc(1, sizeof(Local));
    L->v = v;
    L->c = mk(X->X[3 * n], X->X[3 * n + 1], X->X[3 * n + 2]);
    L->rho = X->R[n];
    for (int m = 1; m <= v; ++m) {
        int s = X->adj[X->off[n] + m - 1];
        int f = X->sa[s] == n ? X->sb[s] : X->sa[s];
        L->sid[m] = s;
        L->far[m] = f;
        if (f == n) { node_fail(R, ST_INVALID_STRUT); continue; }
        V3 cf = mk(X->X[3 * f], X->X[3 * f + 1], X->X[3 * f + 2]);
        V3 d = sub(cf, L->c);
        double len = nrm(d);
        double sig = (L->rho - X->R[f]) / len;
        if (!(len > 0) || !(fabs(sig) < 1.0)) { node_fail(R, ST_INVALID_STRUT); continue; }
        L->len[m] = len;
        L->e[m] = scl(d, 1.0 / len);
        L->sig[m] = sig;
        L->kap[m] = sqrt(1.0 - sig * sig);
        L->g[m] = scl(L->e[m], 1.0 / L->kap[m]);
        L->h[m] = L->rho * sig / L->kap[m];
        int lo = n < f ? (int)n : f, hi = n < f ? f : (int)n;
        L->lower[m] = (n < f);
        V3 clo = mk(X->X[3 * lo], X->X[3 * lo + 1], X->X[3 * lo + 2]);
        V3 chi = mk(X->X[3 * hi], X->X[3 * hi + 1], X->X[3 * hi + 2]);
        L->es[m] = unit(sub(chi, clo));
        L->frame_gap[m] = strut_frame(L->es[m], &L->rh[m], &L->qh[m]);
    }
    for (int m = 1; m <= v; ++m)
        for (int j = m + 1; j <= v; ++j)
            if (L->far[m] == L->far[j]) node_fail(R, ST_DUPLICATE);
    if (R->status) { free(L); return; }

    double margin = 1e300;
    int mkind = 0;
    double kmin[MK_N];
    for (int i = 0; i < MK_N; ++i) kmin[i] = 1e300;
    /* Steps 1-2: conics and their kept arcs */
    int cap = 64, ne = 0;
    Arc *arcs = malloc(sizeof(Arc) * cap);
    RawArc *raw = malloc(sizeof(RawArc) * 2 * (v + 2));
    for (int p = 0; p <= v; ++p)
        for (int q = p + 1; q <= v; ++q) {
            V3 o, a, b;
            if (p == 0) {
                conic_circle(L, q, &o, &a, &b);
            } else {
                double em;
                if (conic_ellipse(L, p, q, &o, &a, &b, &em) < 0) {
                    node_fail(R, ST_NON_ELLIPTIC);
                    continue;
                }
                LOWER(em, MK_ELLIPSE);
            }
            double cm = 1e300;
            int nra = trim_conic(L, p, q, o, a, b, raw, &cm);
            LOWER(cm, MK_CONIC);
            for (int i = 0; i < nra; ++i) {
                if (ne == cap) { cap *= 2; arcs = realloc(arcs, sizeof(Arc) * cap); }
                Arc *A = &arcs[ne++];
                memset(A, 0, sizeof(*A));
                A->p = p; A->q = q; A->o = o; A->a = a; A->b = b;
                A->t1 = raw[i].t1; A->t2 = raw[i].t2;
                A->rs = raw[i].rs; A->re = raw[i].re; A->full = raw[i].full;
                A->contour = -1;
            }
        }
    free(raw);
    if (R->status) { free(arcs); free(L); return; }

    /* Step 3: vertices = arc ends, named by their triple and root rank */
    int vcap = 64, nv = 0;
    Vert *verts = malloc(sizeof(Vert) * vcap);
    for (int i = 0; i < ne; ++i) {
        Arc *A = &arcs[i];
        if (A->full) {
            uint32_t nm = vname(A->p, A->q, 255, 0);
            A->ns = A->ne_ = nm;
            if (nv == vcap) { vcap *= 2; verts = realloc(verts, sizeof(Vert) * vcap); }
            verts[nv].name = nm;
            verts[nv].w = conic_pt(A->o, A->a, A->b, 0.0);
            verts[nv].sep = verts[nv].gap = 1e300;
            ++nv;
            /* the start point of a whole circle depends on the strut frame.
             * An exact tie of |e_s,j| (gap 0: equal magnitudes of the FP32
             * coordinate differences, which FP32 arithmetic keeps equal) is
             * decided by the lowest index on both sides; only a near tie is
             * a margin. */
            if (A->p == 0 && L->frame_gap[A->q] > 0.0) {
                LOWER(L->frame_gap[A->q], MK_FRAME);
            }
            continue;
        }
        for (int end = 0; end < 2; ++end) {
            int r = end ? A->re : A->rs;
            double t = end ? A->t2 : A->t1;
            int tr[3] = {A->p, A->q, r};
            /* sort triple */
            for (int x = 0; x < 2; ++x)
                for (int y = 0; y < 2 - x; ++y)
                    if (tr[y] > tr[y + 1]) { int s = tr[y]; tr[y] = tr[y + 1]; tr[y + 1] = s; }
            V3 roots[2];
            double sep = 0;
            V3 xt = conic_pt(A->o, A->a, A->b, t);
            int nroot = triple_roots(L, tr[0], tr[1], tr[2], roots, &sep);
            int root = 0;
            if (nroot < 2) { node_fail(R, ST_TOPOLOGY); continue; }
            double d0 = nrm(sub(roots[0], xt)), d1 = nrm(sub(roots[1], xt));
            root = d1 < d0 ? 1 : 0;
            if ((root ? d1 : d0) > 1e-6 * L->rho) node_fail(R, ST_TOPOLOGY);
            LOWER(sep, MK_ROOTS);
            uint32_t nm = vname(tr[0], tr[1], tr[2], root);
            if (end) A->ne_ = nm; else A->ns = nm;
            if (find_vert(verts, nv, nm) < 0) {
                if (nv == vcap) { vcap *= 2; verts = realloc(verts, sizeof(Vert) * vcap); }
                verts[nv].name = nm;
                verts[nv].w = roots[root];
                verts[nv].sep = sep;
                ++nv;
                /* gap to the runner-up strut at the tie point */
                double ptie = Pval(L, tr[0], roots[root]);
                double best = -1e300;
                for (int s2 = 0; s2 <= v; ++s2) {
                    if (s2 == tr[0] || s2 == tr[1] || s2 == tr[2]) continue;
                    double ps = Pval(L, s2, roots[root]);
                    if (ps > best) best = ps;
                }
                verts[nv - 1].gap = (ptie - best) / L->rho;
                LOWER((ptie - best) / L->rho, MK_GAP);
            }
        }
    }
    if (R->status) { free(arcs); free(verts); free(L); return; }
    qsort(verts, nv, sizeof(Vert), vert_cmp);
    qsort(arcs, ne, sizeof(Arc), arc_cmp);
    for (int i = 0; i < ne; ++i) {
        arcs[i].vs = find_vert(verts, nv, arcs[i].ns);
        arcs[i].ve = find_vert(verts, nv, arcs[i].ne_);
    }
    /* each real vertex must end exactly three arcs */
    {
        int *deg = calloc(nv, sizeof(int));
        for (int i = 0; i < ne; ++i) {
            if (arcs[i].full) continue;
            deg[arcs[i].vs]++;
            deg[arcs[i].ve]++;
        }
        for (int i = 0; i < nv; ++i)
            if ((verts[i].name & 0xff00u) != 0xff00u && deg[i] != 3) node_fail(R, ST_TOPOLOGY);
        free(deg);
    }

    /* Step 4a: loops per strut end, ordered by the strut-frame angle phi */
    int *loop_off = calloc(v + 1, sizeof(int));
    int *loop_arc = malloc(sizeof(int) * (2 * ne + 1));
    int *loop_dir = malloc(sizeof(int) * (2 * ne + 1));
    int nl = 0;
    {
        int *mine = malloc(sizeof(int) * (ne + 1));
        int *dirs = malloc(sizeof(int) * (ne + 1));
        int *used = malloc(sizeof(int) * (ne + 1));
        for (int m = 1; m <= v; ++m) {
            int cnt = 0, nfull = 0;
            for (int i = 0; i < ne; ++i) {
                if (arcs[i].p != m && arcs[i].q != m) continue;
                Arc *A = &arcs[i];
                double tm = 0.5 * (A->t1 + A->t2);
                V3 w = conic_pt(A->o, A->a, A->b, tm);
                V3 dw = sub(scl(A->a, cos(tm)), scl(A->b, sin(tm)));
                double s = dot(cross(w, dw), L->es[m]);
                dirs[cnt] = s > 0 ? 1 : -1;
                nfull += A->full;
                mine[cnt++] = i;
            }
            loop_off[m - 1] = nl;
            if (cnt == 0 || (nfull && cnt != 1)) { node_fail(R, ST_LOOP); continue; }
            if (nfull) {
                loop_arc[nl] = mine[0]; loop_dir[nl] = dirs[0]; ++nl;
                continue;
            }
            /* start at the arc whose loop-start vertex has the smallest name */
            int first = 0;
            for (int j = 0; j < cnt; ++j) {
                Arc *A = &arcs[mine[j]], *F = &arcs[mine[first]];
                uint32_t sj = dirs[j] > 0 ? A->ns : A->ne_;
                uint32_t sf = dirs[first] > 0 ? F->ns : F->ne_;
                if (sj < sf) first = j;
                used[j] = 0;
            }
            int cur = first, steps = 0;
            while (1) {
                used[cur] = 1;
                loop_arc[nl] = mine[cur]; loop_dir[nl] = dirs[cur]; ++nl; ++steps;
                Arc *A = &arcs[mine[cur]];
                uint32_t endn = dirs[cur] > 0 ? A->ne_ : A->ns;
                int nxt = -1, hits = 0;
                for (int j = 0; j < cnt; ++j) {
                    Arc *B = &arcs[mine[j]];
                    uint32_t sj = dirs[j] > 0 ? B->ns : B->ne_;
                    if (sj == endn) { nxt = j; ++hits; }
                }
                if (hits != 1) { node_fail(R, ST_LOOP); break; }
                if (nxt == first) break;
                if (used[nxt]) { node_fail(R, ST_LOOP); break; }
                cur = nxt;
            }
            if (steps != cnt) node_fail(R, ST_LOOP);
        }
        loop_off[v] = nl;
        free(mine); free(dirs); free(used);
    }

    /* Step 4b: hole contours = connected circular arcs (Sec. 5) */
    int nc = 0;
    {
        int *par = malloc(sizeof(int) * (ne + 1));
        for (int i = 0; i < ne; ++i) par[i] = i;
#define FIND(x) ({ int r_ = (x); while (par[r_] != r_) r_ = par[r_]; r_; })
        for (int i = 0; i < ne; ++i) {
            if (arcs[i].p != 0 || arcs[i].full) continue;
            for (int j = i + 1; j < ne; ++j) {
                if (arcs[j].p != 0 || arcs[j].full) continue;
                if (arcs[i].vs == arcs[j].vs || arcs[i].vs == arcs[j].ve || arcs[i].ve == arcs[j].vs ||
                    arcs[i].ve == arcs[j].ve) {
                    int a = FIND(i), b = FIND(j);
                    if (a != b) par[a < b ? b : a] = a < b ? a : b;
                }
            }
        }
        /* contour order: by the smallest vertex name on it */
        uint32_t *cmin = malloc(sizeof(uint32_t) * (ne + 1));
        int *croot = malloc(sizeof(int) * (ne + 1));
        int nroots = 0;
        for (int i = 0; i < ne; ++i) {
            if (arcs[i].p != 0) continue;
            int r = FIND(i);
            int idx = -1;
            for (int j = 0; j < nroots; ++j)
                if (croot[j] == r) idx = j;
            uint32_t mn = arc_key_name(&arcs[i]);
            if (idx < 0) { croot[nroots] = r; cmin[nroots] = mn; ++nroots; }
            else if (mn < cmin[idx]) cmin[idx] = mn;
        }
#undef FIND
        /* rank contours by cmin */
        for (int i = 0; i < ne; ++i) {
            if (arcs[i].p != 0) continue;
            int r = i;
            while (par[r] != r) r = par[r];
            int idx = 0;
            for (int j = 0; j < nroots; ++j)
                if (croot[j] == r) idx = j;
            int rank = 0;
            for (int j = 0; j < nroots; ++j)
                if (cmin[j] < cmin[idx]) ++rank;
            arcs[i].contour = rank;
        }
        nc = nroots;
        /* every vertex on a contour joins exactly two circular arcs */
        int *cdeg = calloc(nv, sizeof(int));
        for (int i = 0; i < ne; ++i)
            if (arcs[i].p == 0 && !arcs[i].full) { cdeg[arcs[i].vs]++; cdeg[arcs[i].ve]++; }
        for (int i = 0; i < nv; ++i)
            if (cdeg[i] != 0 && cdeg[i] != 2) node_fail(R, ST_TOPOLOGY);
        free(cdeg); free(par); free(cmin); free(croot);
    }
    /* Euler relation of the arrangement on the node sphere: V - E + C = 2 - v
     * (fails for annular holes, which a barycentre fan cannot fill). */
    if (nv - ne + nc != 2 - v) node_fail(R, ST_TOPOLOGY);

    R->nv = nv; R->ne = ne; R->nc = nc;
    R->verts = verts; R->arcs = arcs;
    R->loop_off = loop_off; R->loop_arc = loop_arc; R->loop_dir = loop_dir;
    if (R->status) {
        R->margin = margin;
        R->margin_kind = mkind;
        memcpy(R->kmargin, kmin, sizeof(kmin));
        free(L);
        return;
    }

    /* Step 5: subdivision at resolution k (Eqs. 11-12) */
    int k = X->k;
    int nmesh = nv;
    for (int i = 0; i < ne; ++i) {
        Arc *A = &arcs[i];
        if (A->full) {
            A->nseg = k;
        } else {
            double u = k * (A->t2 - A->t1) / TWO_PI;
            double fl = floor(u);
            int ns = (int)fl + 1;
            A->nseg = ns < k ? ns : k;
            LOWER(fmin(u - fl, fl + 1 - u), MK_FLOOR);
        }
        A->mbase = nmesh;
        nmesh += A->nseg - 1;
    }
    int cbase = nmesh;
    nmesh += nc;
    double *mw = malloc(sizeof(double) * 3 * (nmesh + 1));
    for (int i = 0; i < nv; ++i) {
        mw[3 * i] = verts[i].w.x; mw[3 * i + 1] = verts[i].w.y; mw[3 * i + 2] = verts[i].w.z;
    }
    for (int i = 0; i < ne; ++i) {
        Arc *A = &arcs[i];
        int fwd = A->full || A->ns <= A->ne_;
        for (int j = 0; j < A->nseg - 1; ++j) {
            int ii = fwd ? j + 1 : A->nseg - 1 - j; /* Eq. 12 index */
            double s = A->t1 + (A->t2 - A->t1) * ii / A->nseg;
            V3 w = conic_pt(A->o, A->a, A->b, s);
            int m = A->mbase + j;
            mw[3 * m] = w.x; mw[3 * m + 1] = w.y; mw[3 * m + 2] = w.z;
        }
    }
    /* local mesh index of the interior point with Eq. 12 index ii on arc A */
#define INTERIOR(A, ii) ((A)->mbase + (((A)->full || (A)->ns <= (A)->ne_) ? (ii) - 1 : (A)->nseg - 1 - (ii)))
    /* Eq. 13 hole centres */
    double *cb = calloc(3 * (nc + 1), sizeof(double));
    {
        int *cntv = calloc(nc + 1, sizeof(int));
        V3 *sum = calloc(nc + 1, sizeof(V3));
        char *seen = calloc(nv + 1, 1);
        for (int c = 0; c < nc; ++c) {
            memset(seen, 0, nv + 1);
            for (int i = 0; i < ne; ++i) {
                Arc *A = &arcs[i];
                if (A->p != 0 || A->contour != c) continue;
                int ends[2] = {A->vs, A->ve};
                for (int t = 0; t < 2; ++t)
                    if (!seen[ends[t]]) {
                        seen[ends[t]] = 1;
                        sum[c] = add(sum[c], verts[ends[t]].w);
                        cntv[c]++;
                    }
                for (int j = 0; j < A->nseg - 1; ++j) {
                    int m = A->mbase + j;
                    sum[c] = add(sum[c], mk(mw[3 * m], mw[3 * m + 1], mw[3 * m + 2]));
                    cntv[c]++;
                }
            }
            /* Eq. 13: barycentre of the contour vertices, projected onto the
             * nodal sphere.  When the barycentre is within 1e-3 rho of the
             * centre (cylindrical free ends) its direction is noise, so the
             * direction -sum(e_m) is used; if the projected point falls under a
             * strut (holes larger than a hemisphere), the opposite point is
             * taken, so the fan apex always lies on the hole. */
            V3 bc = scl(sum[c], 1.0 / cntv[c]);
            double bl = nrm(bc);
            LOWER(fabs(bl / L->rho - 1e-3), MK_HOLE);
            V3 dir;
            if (bl >= 1e-3 * L->rho) {
                dir = scl(bc, 1.0 / bl);
            } else {
                V3 se = mk(0, 0, 0);
                for (int m = 1; m <= v; ++m) se = add(se, L->e[m]);
                if (nrm(se) < 1e-3) { node_fail(R, ST_TOPOLOGY); dir = mk(0, 0, 1); }
                else dir = scl(unit(se), -1.0);
            }
            double pm = -1e300;
            for (int m = 1; m <= v; ++m) {
                double pv = Pval(L, m, scl(dir, L->rho));
                if (pv > pm) pm = pv;
            }
            LOWER(fabs(pm) / L->rho, MK_HOLE);
            if (pm > 0) {
                dir = scl(dir, -1.0);
                pm = -1e300;
                for (int m = 1; m <= v; ++m) {
                    double pv = Pval(L, m, scl(dir, L->rho));
                    if (pv > pm) pm = pv;
                }
                LOWER(fabs(pm) / L->rho, MK_HOLE);
                if (pm > 0) node_fail(R, ST_TOPOLOGY);
            }
            V3 bp = scl(dir, L->rho);
            int m = cbase + c;
            mw[3 * m] = bp.x; mw[3 * m + 1] = bp.y; mw[3 * m + 2] = bp.z;
            cb[3 * c] = bp.x; cb[3 * c + 1] = bp.y; cb[3 * c + 2] = bp.z;
        }
        free(cntv); free(sum); free(seen);
    }
    /* fans: one triangle per circular-arc segment, oriented so the shared edge
     * runs opposite to the strut band's copy of it */
    int nfan = 0;
    for (int i = 0; i < ne; ++i)
        if (arcs[i].p == 0) nfan += arcs[i].nseg;
    int *fan = malloc(sizeof(int) * 3 * (nfan + 1));
    {
        int f = 0;
        for (int i = 0; i < ne; ++i) {
            Arc *A = &arcs[i];
            if (A->p != 0) continue;
            int fwd = A->full || A->ns <= A->ne_;
            int lower = L->lower[A->q];
            for (int j = 0; j < A->nseg; ++j) {
                /* canonical segment j joins canonical points j and j+1; map to
                 * Eq. 12 indices then order them by increasing t (= phi). */
                int i0 = fwd ? j : A->nseg - j, i1 = fwd ? j + 1 : A->nseg - j - 1;
                int lo_i = i0 < i1 ? i0 : i1, hi_i = i0 < i1 ? i1 : i0;
                int u, u2;
                u = lo_i == 0 ? A->vs : INTERIOR(A, lo_i);
                u2 = hi_i == A->nseg ? A->ve : INTERIOR(A, hi_i);
                int ctr = cbase + A->contour;
                fan[3 * f] = ctr;
                if (lower) { fan[3 * f + 1] = u2; fan[3 * f + 2] = u; }
                else { fan[3 * f + 1] = u; fan[3 * f + 2] = u2; }
                ++f;
            }
        }
    }
    /* loop vertex sequences with strut-frame angles */
    int *lv_off = calloc(v + 1, sizeof(int));
    int tot = 0;
    for (int li = 0; li < nl; ++li) tot += arcs[loop_arc[li]].nseg;
    int *lv_idx = malloc(sizeof(int) * (tot + 1));
    double *lv_phi = malloc(sizeof(double) * (tot + 1));
    uint8_t *lv_whole = malloc(tot + 1);
    {
        int pos = 0;
        for (int m = 1; m <= v; ++m) {
            lv_off[m - 1] = pos;
            int b0 = pos;
            for (int li = loop_off[m - 1]; li < loop_off[m]; ++li) {
                Arc *A = &arcs[loop_arc[li]];
                int d = loop_dir[li];
                /* loop-start vertex then interior points in loop direction;
                 * on a tangency circle phi is the circle parameter itself
                 * (the circle is parametrised in the strut frame), elsewhere
                 * it is measured from the point */
                for (int j = 0; j < A->nseg; ++j) {
                    int ii = d > 0 ? j : A->nseg - j;
                    int mi = j == 0 ? (d > 0 ? A->vs : A->ve) : INTERIOR(A, ii);
                    lv_idx[pos] = mi;
                    lv_whole[pos] = (uint8_t)(A->p == 0 && A->full);
                    if (A->p == 0) {
                        double t = A->t1 + (A->t2 - A->t1) * ii / A->nseg;
                        if (t >= TWO_PI) t -= TWO_PI;
                        if (t > M_PI) t -= TWO_PI;
                        lv_phi[pos] = t;
                    } else {
                        lv_phi[pos] = phi_of(L, m, mk(mw[3 * mi], mw[3 * mi + 1], mw[3 * mi + 2]));
                    }
                    ++pos;
                }
            }
            /* the loop must be a graph over phi: strictly increasing, one turn */
            double wind = 0.0, minstep = 1e300;
            int cnt = pos - b0;
            for (int i = 0; i < cnt; ++i) {
                double dphi = wrap_pi(lv_phi[b0 + (i + 1) % cnt] - lv_phi[b0 + i]);
                if (cnt == 1) dphi = TWO_PI;
                wind += dphi;
                if (dphi < minstep) minstep = dphi;
            }
            if (!(minstep > 0) || fabs(wind - TWO_PI) > 1e-6) node_fail(R, ST_LOOP);
            LOWER(minstep, MK_STEP);
        }
        lv_off[v] = pos;
    }
#undef INTERIOR
    R->nmesh = nmesh; R->nfan = nfan; R->mesh_w = mw; R->fan = fan;
    R->lv_off = lv_off; R->lv_idx = lv_idx; R->lv_phi = lv_phi; R->lv_whole = lv_whole; R->cont_b = cb;
    R->margin = margin;
    R->margin_kind = mkind;
    memcpy(R->kmargin, kmin, sizeof(kmin));
    free(L);
}

/* ------------------------------------------------------------------ */
/* strut bands: phi-merge zipper (Sec. 5)                               */

/* cyclic predecessor: the element of Y with the largest key below (phi, tag);
 * keys compare (phi, tag) lexicographically, tag 0 for the lower end's loop */
static int pred(const double *phy, int ny, int tagy, double phx, int tagx)
{
    int best = -1, top = 0;
    for (int i = 0; i < ny; ++i) {
        int lt = phy[i] < phx || (phy[i] == phx && tagy < tagx);
        if (lt && (best < 0 || phy[i] > phy[best] || (phy[i] == phy[best] && i > best))) best = i;
        if (phy[i] > phy[top]) top = i;
    }
    return best >= 0 ? best : top;
}

static void strut_band(Ctx *X, int64_t s)
{
    int64_t a = X->sa[s] < X->sb[s] ? X->sa[s] : X->sb[s];
    int64_t b = X->sa[s] < X->sb[s] ? X->sb[s] : X->sa[s];
    NodeRes *Ra = &X->nodes[a], *Rb = &X->nodes[b];
    int64_t *T = X->tri + 3 * X->band_off[s];
    if (X->band_off[s + 1] == X->band_off[s]) return;
    int ma = -1, mb = -1;
    for (int m = 1; m <= Ra->v; ++m)
        if (X->adj[X->off[a] + m - 1] == s) ma = m;
    for (int m = 1; m <= Rb->v; ++m)
        if (X->adj[X->off[b] + m - 1] == s) mb = m;
    int na = Ra->lv_off[ma] - Ra->lv_off[ma - 1], nb = Rb->lv_off[mb] - Rb->lv_off[mb - 1];
    const int *ia = Ra->lv_idx + Ra->lv_off[ma - 1], *ib = Rb->lv_idx + Rb->lv_off[mb - 1];
    const double *pa = Ra->lv_phi + Ra->lv_off[ma - 1], *pb = Rb->lv_phi + Rb->lv_off[mb - 1];
    int64_t oa = X->mesh_off[a], ob = X->mesh_off[b];
    int t = 0;
    for (int i = 0; i < na; ++i) {
        int i2 = (i + 1) % na;
        int ap = pred(pb, nb, 1, pa[i2], 0);
        T[3 * t] = oa + ia[i]; T[3 * t + 1] = oa + ia[i2]; T[3 * t + 2] = ob + ib[ap];
        ++t;
    }
    for (int j = 0; j < nb; ++j) {
        int j2 = (j + 1) % nb;
        int ap = pred(pa, na, 0, pb[j2], 1);
        T[3 * t] = ob + ib[j2]; T[3 * t + 1] = ob + ib[j]; T[3 * t + 2] = oa + ia[ap];
        ++t;
    }
    /* margin: the smallest phi gap between the two loops' samples.  Two
     * samples of whole tangency circles are both at t = 2 pi i / k (phi is
     * the circle parameter, the same sub-parameters at both ends): they tie
     * exactly or lie a step apart, and an exact tie is decided by the end
     * tag on both sides, so such pairs are no margin. */
    const uint8_t *wa = Ra->lv_whole + Ra->lv_off[ma - 1], *wb = Rb->lv_whole + Rb->lv_off[mb - 1];
    double mg = 1e300;
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
            if (wa[i] && wb[j]) continue;
            double d = fabs(wrap_pi(pa[i] - pb[j]));
            if (d < mg) mg = d;
        }
    X->strut_margin[s] = mg;
}

/* ------------------------------------------------------------------ */
/* threading                                                            */

typedef struct {
    Ctx *X;
    int phase;
} Job;

static void *worker(void *arg)
{
    Job *J = arg;
    Ctx *X = J->X;
    int64_t total = J->phase == 0 ? X->N : X->S;
    const int64_t chunk = 64;
    while (1) {
        int64_t i0 = __atomic_fetch_add(&X->next, chunk, __ATOMIC_RELAXED);
        if (i0 >= total) break;
        int64_t i1 = i0 + chunk < total ? i0 + chunk : total;
        for (int64_t i = i0; i < i1; ++i) {
            if (J->phase == 0) node_compute(X, i);
            else strut_band(X, i);
        }
    }
    return NULL;
}

static void run_phase(Ctx *X, int phase)
{
    X->next = 0;
    int nt = X->nthreads > 0 ? X->nthreads : 1;
    pthread_t th[256];
    Job J = {X, phase};
    if (nt > 256) nt = 256;
    for (int i = 0; i < nt; ++i) pthread_create(&th[i], NULL, worker, &J);
    for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------------ */
/* public entry points (loaded with ctypes by the tests)                */

void orc_free(Ctx *X);

/* Runs the whole method on a lattice given as FP64 arrays (used directly
 * for finite differences).  Returns NULL on bad arguments (indices out of
 * range). */
Ctx *orc_run_f64(int64_t N, int64_t S, const double *x, const double *y, const double *z, const double *rad,
                 const int32_t *sa, const int32_t *sb, int k, int nthreads)
{
    if (N < 0 || S < 0 || k < 1) return NULL;
    for (int64_t s = 0; s < S; ++s)
        if (sa[s] < 0 || sa[s] >= N || sb[s] < 0 || sb[s] >= N) return NULL;
    Ctx *X = calloc(1, sizeof(Ctx));
    X->N = N; X->S = S; X->k = k; X->nthreads = nthreads;
    double *XX = malloc(sizeof(double) * 3 * (N + 1));
    double *RR = malloc(sizeof(double) * (N + 1));
    for (int64_t i = 0; i < N; ++i) {
        XX[3 * i] = x[i]; XX[3 * i + 1] = y[i]; XX[3 * i + 2] = z[i];
        RR[i] = rad[i];
    }
    X->X = XX; X->R = RR; X->sa = sa; X->sb = sb;
    /* adjacency lists, incident struts in increasing strut id */
    X->off = calloc(N + 1, sizeof(int64_t));
    for (int64_t s = 0; s < S; ++s) {
        X->off[sa[s] + 1]++;
        if (sb[s] != sa[s]) X->off[sb[s] + 1]++;
    }
    for (int64_t i = 0; i < N; ++i) X->off[i + 1] += X->off[i];
    X->adj = malloc(sizeof(int32_t) * (X->off[N] + 1));
    int64_t *fill = malloc(sizeof(int64_t) * (N + 1));
    memcpy(fill, X->off, sizeof(int64_t) * N);
    for (int64_t s = 0; s < S; ++s) {
        X->adj[fill[sa[s]]++] = (int32_t)s;
        if (sb[s] != sa[s]) X->adj[fill[sb[s]]++] = (int32_t)s;
    }
    free(fill);
    X->nodes = calloc(N + 1, sizeof(NodeRes));
    run_phase(X, 0);
    /* mesh vertex / triangle numbering */
    X->mesh_off = calloc(N + 1, sizeof(int64_t));
    X->fan_off = calloc(N + 1, sizeof(int64_t));
    X->band_off = calloc(S + 1, sizeof(int64_t));
    X->strut_margin = malloc(sizeof(double) * (S + 1));
    X->strut_status = calloc(S + 1, sizeof(int));
    for (int64_t i = 0; i < N; ++i) {
        NodeRes *R = &X->nodes[i];
        int ok = R->status == 0;
        X->mesh_off[i + 1] = X->mesh_off[i] + (ok ? R->nmesh : 0);
        X->fan_off[i + 1] = X->fan_off[i] + (ok ? R->nfan : 0);
    }
    for (int64_t s = 0; s < S; ++s) {
        X->strut_margin[s] = 1e300;
        int64_t a = sa[s], b = sb[s];
        NodeRes *Ra = &X->nodes[a], *Rb = &X->nodes[b];
        int64_t cnt = 0;
        if (Ra->status == 0 && Rb->status == 0 && a != b) {
            for (int m = 1; m <= Ra->v; ++m)
                if (X->adj[X->off[a] + m - 1] == s) cnt += Ra->lv_off[m] - Ra->lv_off[m - 1];
            for (int m = 1; m <= Rb->v; ++m)
                if (X->adj[X->off[b] + m - 1] == s) cnt += Rb->lv_off[m] - Rb->lv_off[m - 1];
        } else {
            X->strut_status[s] = 1;
        }
        X->band_off[s + 1] = X->band_off[s] + cnt;
    }
    X->n_mesh = X->mesh_off[N];
    X->n_band = X->band_off[S];
    X->n_fan = X->fan_off[N];
    X->mesh = malloc(sizeof(double) * 3 * (X->n_mesh + 1));
    X->tri = malloc(sizeof(int64_t) * 3 * (X->n_band + X->n_fan + 1));
    for (int64_t i = 0; i < N; ++i) {
        NodeRes *R = &X->nodes[i];
        if (R->status) continue;
        double *dst = X->mesh + 3 * X->mesh_off[i];
        for (int j = 0; j < R->nmesh; ++j) {
            dst[3 * j] = XX[3 * i] + R->mesh_w[3 * j];
            dst[3 * j + 1] = XX[3 * i + 1] + R->mesh_w[3 * j + 1];
            dst[3 * j + 2] = XX[3 * i + 2] + R->mesh_w[3 * j + 2];
        }
        int64_t *T = X->tri + 3 * (X->n_band + X->fan_off[i]);
        for (int j = 0; j < 3 * R->nfan; ++j) T[j] = X->mesh_off[i] + R->fan[j];
    }
    run_phase(X, 1);
    return X;
}

/* The same on a lattice given as FP32 arrays (promoted to FP64). */
Ctx *orc_run(int64_t N, int64_t S, const float *x, const float *y, const float *z, const float *rad,
             const int32_t *sa, const int32_t *sb, int k, int nthreads)
{
    if (N < 0) return NULL;
    double *d = malloc(sizeof(double) * 4 * (N + 1));
    for (int64_t i = 0; i < N; ++i) {
        d[i] = x[i];
        d[(N + 1) + i] = y[i];
        d[2 * (N + 1) + i] = z[i];
        d[3 * (N + 1) + i] = rad[i];
    }
    Ctx *X = orc_run_f64(N, S, d, d + (N + 1), d + 2 * (N + 1), d + 3 * (N + 1), sa, sb, k, nthreads);
    free(d);
    return X;
}

void orc_free(Ctx *X)
{
    if (!X) return;
    for (int64_t i = 0; i < X->N; ++i) {
        NodeRes *R = &X->nodes[i];
        free(R->verts); free(R->arcs); free(R->loop_off); free(R->loop_arc); free(R->loop_dir);
        free(R->mesh_w); free(R->fan); free(R->lv_off); free(R->lv_idx); free(R->lv_phi); free(R->lv_whole);
        free(R->cont_b);
    }
    free(X->nodes); free(X->off); free(X->adj); free((void *)X->X); free((void *)X->R);
    free(X->mesh_off); free(X->band_off); free(X->fan_off); free(X->mesh); free(X->tri);
    free(X->strut_margin); free(X->strut_status);
    free(X);
}

/* sizes: [n_vertices, n_arcs, n_contours, n_mesh, n_band, n_fan, n_loop_entries] */
void orc_sizes(const Ctx *X, int64_t *out)
{
    int64_t nv = 0, ne = 0, nc = 0, nl = 0;
    for (int64_t i = 0; i < X->N; ++i) {
        const NodeRes *R = &X->nodes[i];
        nv += R->nv; ne += R->ne; nc += R->nc;
        if (R->loop_off) nl += R->loop_off[R->v];
    }
    out[0] = nv; out[1] = ne; out[2] = nc;
    out[3] = X->n_mesh; out[4] = X->n_band; out[5] = X->n_fan; out[6] = nl;
}

/* per node: status, valence, nv, ne, nc, nmesh, nfan, margin kind (int32 x 8)
 * and margin */
void orc_nodes(const Ctx *X, int32_t *cnt, double *margin)
{
    for (int64_t i = 0; i < X->N; ++i) {
        const NodeRes *R = &X->nodes[i];
        int32_t *c = cnt + 8 * i;
        c[0] = R->status; c[1] = R->v; c[2] = R->nv; c[3] = R->ne; c[4] = R->nc;
        c[5] = R->status ? 0 : R->nmesh; c[6] = R->status ? 0 : R->nfan; c[7] = R->margin_kind;
        margin[i] = R->margin;
    }
}

/* per node: the smallest margin of each kind MK_* = 1..8 (double x 8; 1e300
 * where a kind did not occur) */
void orc_node_margins(const Ctx *X, double *out)
{
    for (int64_t i = 0; i < X->N; ++i)
        for (int kd = 1; kd < MK_N; ++kd) out[8 * i + kd - 1] = X->nodes[i].kmargin[kd];
}

/* meta-mesh vertices, concatenated in node order: name, local position,
 * conditioning (root separation, runner-up gap; both in units of rho) */
void orc_vertices(const Ctx *X, uint32_t *name, double *w, double *cond)
{
    int64_t o = 0;
    for (int64_t i = 0; i < X->N; ++i) {
        const NodeRes *R = &X->nodes[i];
        for (int j = 0; j < R->nv; ++j, ++o) {
            name[o] = R->verts[j].name;
            cond[2 * o] = R->verts[j].sep;
            cond[2 * o + 1] = R->verts[j].gap;
            w[3 * o] = R->verts[j].w.x; w[3 * o + 1] = R->verts[j].w.y; w[3 * o + 2] = R->verts[j].w.z;
        }
    }
}

/* arcs in node order: ints (p, q, vs, ve, nseg, contour, full) and doubles
 * (o[3], a[3], b[3], t1, t2), positions local to the node */
void orc_arcs(const Ctx *X, int32_t *iv, double *dv)
{
    int64_t o = 0;
    for (int64_t i = 0; i < X->N; ++i) {
        const NodeRes *R = &X->nodes[i];
        for (int j = 0; j < R->ne; ++j, ++o) {
            const Arc *A = &R->arcs[j];
            int32_t *I = iv + 7 * o;
            double *D = dv + 11 * o;
            I[0] = A->p; I[1] = A->q; I[2] = A->vs; I[3] = A->ve; I[4] = A->nseg;
            I[5] = A->contour; I[6] = A->full;
            D[0] = A->o.x; D[1] = A->o.y; D[2] = A->o.z;
            D[3] = A->a.x; D[4] = A->a.y; D[5] = A->a.z;
            D[6] = A->b.x; D[7] = A->b.y; D[8] = A->b.z;
            D[9] = A->t1; D[10] = A->t2;
        }
    }
}

/* loops per half-edge in adjacency order: offsets (2S+1) and (arc, dir);
 * arc indices are local to the node */
void orc_loops(const Ctx *X, int64_t *off, int32_t *arc, int32_t *dir)
{
    int64_t o = 0, h = 0;
    for (int64_t i = 0; i < X->N; ++i) {
        const NodeRes *R = &X->nodes[i];
        for (int m = 1; m <= R->v; ++m) {
            off[h++] = o;
            if (!R->loop_off) continue;
            for (int j = R->loop_off[m - 1]; j < R->loop_off[m]; ++j, ++o) {
                arc[o] = R->loop_arc[j];
                dir[o] = R->loop_dir[j];
            }
        }
    }
    off[h] = o;
}

/* adjacency (strut ids per node in label order) */
void orc_adjacency(const Ctx *X, int64_t *off, int32_t *adj)
{
    memcpy(off, X->off, sizeof(int64_t) * (X->N + 1));
    memcpy(adj, X->adj, sizeof(int32_t) * X->off[X->N]);
}

/* mesh: absolute vertices, triangles, per-node mesh offsets, per-strut band
 * offsets, per-node fan offsets (fans follow all bands), strut margins */
void orc_mesh(const Ctx *X, double *verts, int64_t *tris, int64_t *mesh_off, int64_t *band_off, int64_t *fan_off,
              double *strut_margin, int32_t *strut_status)
{
    memcpy(verts, X->mesh, sizeof(double) * 3 * X->n_mesh);
    memcpy(tris, X->tri, sizeof(int64_t) * 3 * (X->n_band + X->n_fan));
    memcpy(mesh_off, X->mesh_off, sizeof(int64_t) * (X->N + 1));
    memcpy(band_off, X->band_off, sizeof(int64_t) * (X->S + 1));
    memcpy(fan_off, X->fan_off, sizeof(int64_t) * (X->N + 1));
    memcpy(strut_margin, X->strut_margin, sizeof(double) * X->S);
    memcpy(strut_status, X->strut_status, sizeof(int32_t) * X->S);
}

/* Stand-alone Eq. 7 ellipse for tests: node centre c, radius r0; strut p to
 * (cp, rp); strut q to (cq, rq).  out: o[3], a[3], b[3] local to c.
 * Returns -1 if the section is not an ellipse. */
int orc_ellipse(const double *c, double r0, const double *cp, double rp, const double *cq, double rq, double *out)
{
    Local *L = calloc(1, sizeof(Local));
    L->v = 2; L->c = mk(c[0], c[1], c[2]); L->rho = r0;
    const double *cs[2] = {cp, cq};
    double rs[2] = {rp, rq};
    for (int m = 1; m <= 2; ++m) {
        V3 d = sub(mk(cs[m - 1][0], cs[m - 1][1], cs[m - 1][2]), L->c);
        double len = nrm(d);
        L->e[m] = scl(d, 1.0 / len);
        L->sig[m] = (r0 - rs[m - 1]) / len;
        L->kap[m] = sqrt(1 - L->sig[m] * L->sig[m]);
        L->g[m] = scl(L->e[m], 1.0 / L->kap[m]);
        L->h[m] = r0 * L->sig[m] / L->kap[m];
    }
    V3 o, a, b;
    double em;
    int rc = conic_ellipse(L, 1, 2, &o, &a, &b, &em);
    out[0] = o.x; out[1] = o.y; out[2] = o.z;
    out[3] = a.x; out[4] = a.y; out[5] = a.z;
    out[6] = b.x; out[7] = b.y; out[8] = b.z;
    free(L);
    return rc;
}
