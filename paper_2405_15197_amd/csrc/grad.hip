// Adjoint of the triangulation at fixed topology.
//
// Loss terms over the triangle mesh (Area, the volume enclosed about a fixed
// point p0, and the sum of squared vertex norms) and their gradient with
// respect to the mesh vertices; then, per node, the gradient of the loss
// with respect to the node centres and nodal-sphere radii, propagated back
// through the node's mesh vertices while the discrete structure (labels,
// arcs, segment counts, triangles) stays that of the forward pass:
//
//   hole centre (Eq. 13)  rho * b / |b|, b the mean of the contour vertices;
//   interior point (Eq. 12)  o + a sin t_i + b cos t_i, t_i = t1 + (t2 - t1) i / N;
//   arc ends  t1, t2 are the conic parameters of the arc's end vertices;
//   conic (o, a, b)  the tangency circle or the Eq. 7 ellipse of struts p, q;
//   vertex  the tie P_p = P_q = P_r, |w|^2 - rho^2 = P_p^2 (Sec. 4.3.1),
//           differentiated implicitly;
//   strut table  g_m, h_m, e_m from the two node centres and radii.
//
// Conics and strut-table entries are differentiated in forward mode with
// dual numbers (one input direction at a time), everything else in reverse.
#include "geom.h"

namespace lm {
namespace geo {

// Dual number: value and derivative along one input direction.
struct Dual {
    float v, d;
    __device__ Dual() : v(0.f), d(0.f) {}
    __device__ Dual(double x) : v((float)x), d(0.f) {}
    __device__ Dual(float x) : v(x), d(0.f) {}
    __device__ Dual(int x) : v((float)x), d(0.f) {}
    __device__ Dual(float x, float dx) : v(x), d(dx) {}
};
__device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline Dual operator/(Dual a, Dual b)
{
    const float q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
__device__ inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
__device__ inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
__device__ inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
__device__ inline Dual m_sqrt(Dual a)
{
    const float r = sqrtf(a.v);
    return Dual(r, r > 0.f ? 0.5f * a.d / r : 0.f);
}
__device__ inline Dual m_abs(Dual a) { return a.v < 0.f ? -a : a; }
__device__ inline Dual m_max(Dual a, Dual b) { return a.v >= b.v ? a : b; }

}  // namespace geo

namespace {

using namespace geo;

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// loss terms and their gradient with respect to the mesh vertices

__device__ inline float3 f3(const float *p) { return make_float3(p[0], p[1], p[2]); }
__device__ inline float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline float3 crs3(float3 a, float3 b)
{
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ inline void add3(float *p, float3 v, float s)
{
    atomicAdd(p, v.x * s);
    atomicAdd(p + 1, v.y * s);
    atomicAdd(p + 2, v.z * s);
}

// Triangle terms: area 1/2 |N| with N = (b - a) x (c - a), dA/da =
// 1/2 n x (c - b) (cyclic); volume (a' . (b' x c')) / 6 about p0,
// dV/da = (b' x c') / 6.
// Per node (one wave): the gradient of the loss with respect to the node's
// own mesh vertices, gathered over the triangles that touch them (its hole
// fans and the bands of its incident struts) in LDS and written once; the
// loss terms count each band at its lower end node and each fan at its
// node.  Nodes with more mesh vertices than the LDS holds add through
// global atomics instead.
constexpr int kLossLds = 1024;

struct LParams {
    Inputs in;
    Work w;
    const int32_t *tri;
    const float *xyz;
    int64_t cap_mesh, cap_tri;  // sizes of tri / xyz (and dldx) in rows
    float3 p0;
    float w_area, w_vol, w_sq;
    float *dldx;
    double *terms;
};

__global__ void __launch_bounds__(64) k_loss_node(LParams P)
{
    __shared__ float g[kLossLds][3];
    __shared__ double s_terms[3];
    const Work &W = P.w;
    const int64_t N = P.in.n_nodes, S = P.in.n_struts;
    const int64_t n = blockIdx.x;
    const int lane = threadIdx.x;
    if (n >= N) return;
    const int64_t Np1 = N + 1;
    double *nt = W.loss_node + 3 * n;  // this node's share of the loss terms
    // the mesh of the last pass must be complete and fit the buffers given
    // here (tri, xyz and dldx): otherwise nothing is read or written
    const int64_t m_all = W.node_off[(int64_t)NC_MESH * Np1 + N];
    const int64_t t_all = W.band_off[S] + W.node_off[(int64_t)NC_FAN * Np1 + N];
    if ((W.flags[0] & (DF_CAPACITY | DF_RECCAP)) || m_all > P.cap_mesh || t_all > P.cap_tri) {
        if (lane == 0) {
            atomicOr(&W.flags[0], DF_CAPACITY);
            nt[0] = nt[1] = nt[2] = 0.0;
        }
        return;
    }
    const int64_t m0 = W.node_off[(int64_t)NC_MESH * Np1 + n], m1 = W.node_off[(int64_t)NC_MESH * Np1 + n + 1];
    const int M = (int)(m1 - m0);
    if (M == 0) {
        if (lane == 0) nt[0] = nt[1] = nt[2] = 0.0;
        return;
    }
    const bool lds = M <= kLossLds;
    for (int i = lane; i < (lds ? M : 0); i += 64) g[i][0] = g[i][1] = g[i][2] = 0.f;
    if (lane < 3) s_terms[lane] = 0.0;
    __syncthreads();
    double area = 0.0, vol = 0.0, sq = 0.0;
    auto add = [&](int32_t vi, float3 d, float sc) {
        if (vi < m0 || vi >= m1) return;
        if (lds) {
            atomicAdd(&g[vi - m0][0], d.x * sc);
            atomicAdd(&g[vi - m0][1], d.y * sc);
            atomicAdd(&g[vi - m0][2], d.z * sc);
        } else {
            add3(P.dldx + 3 * (int64_t)vi, d, sc);
        }
    };
    // one triangle: gradient on this node's corners; terms when counted here
    auto tri_do = [&](int64_t t, bool count) {
        const int32_t i0 = P.tri[3 * t], i1 = P.tri[3 * t + 1], i2 = P.tri[3 * t + 2];
        const float3 a = sub3(f3(P.xyz + 3 * (int64_t)i0), P.p0), b = sub3(f3(P.xyz + 3 * (int64_t)i1), P.p0),
                     c = sub3(f3(P.xyz + 3 * (int64_t)i2), P.p0);
        const float3 Nn = crs3(sub3(b, a), sub3(c, a));
        const float nl = sqrtf(Nn.x * Nn.x + Nn.y * Nn.y + Nn.z * Nn.z);
        const float3 bc = crs3(b, c), ca = crs3(c, a), ab = crs3(a, b);
        if (count) {
            area += 0.5 * (double)nl;
            vol += ((double)a.x * bc.x + (double)a.y * bc.y + (double)a.z * bc.z) / 6.0;
        }
        // both terms' gradients summed per corner first: one add per corner
        // (same-address LDS atomics of neighbouring lanes serialise)
        const float wa = (P.w_area != 0.f && nl > 0.f) ? 0.5f * P.w_area / nl : 0.f, wv = P.w_vol / 6.f;
        auto corner = [&](float3 e, float3 vterm) {
            const float3 ga = crs3(Nn, e);
            return make_float3(wa * ga.x + wv * vterm.x, wa * ga.y + wv * vterm.y, wa * ga.z + wv * vterm.z);
        };
        if (P.w_area != 0.f || P.w_vol != 0.f) {
            add(i0, corner(sub3(c, b), bc), 1.f);
            add(i1, corner(sub3(a, c), ca), 1.f);
            add(i2, corner(sub3(b, a), ab), 1.f);
        }
    };
    // hole fans of the node
    const int64_t f0 = W.band_off[S] + W.node_off[(int64_t)NC_FAN * Np1 + n];
    const int64_t f1 = W.band_off[S] + W.node_off[(int64_t)NC_FAN * Np1 + n + 1];
    for (int64_t t = f0 + lane; t < f1; t += 64) tri_do(t, true);
    // bands of the incident struts (terms at the lower end)
    const int64_t r0 = W.row[n], r1 = W.row[n + 1];
    for (int64_t h = r0; h < r1; ++h) {
        const int2 he = W.he[h];
        const int64_t b0 = W.band_off[he.y], b1 = W.band_off[he.y + 1];
        const bool lower = (int64_t)he.x > n;
        // even triangles on the first lanes, odd ones after: neighbouring
        // lanes then share fewer corners
        const int64_t nb = b1 - b0, half = (nb + 1) / 2;
        for (int64_t l = lane; l < nb; l += 64) tri_do(b0 + (l < half ? 2 * l : 2 * (l - half) + 1), lower);
    }
    // sum of squared norms over the node's vertices
    for (int i = lane; i < M; i += 64) {
        const float3 x = f3(P.xyz + 3 * (m0 + i));
        sq += (double)x.x * x.x + (double)x.y * x.y + (double)x.z * x.z;
    }
    for (int o = 32; o > 0; o >>= 1) {
        area += __shfl_xor(area, o, 64);
        vol += __shfl_xor(vol, o, 64);
        sq += __shfl_xor(sq, o, 64);
    }
    __syncthreads();
    for (int i = lane; i < M; i += 64) {
        const float3 x = f3(P.xyz + 3 * (m0 + i));
        float *d = P.dldx + 3 * (m0 + i);
        if (lds) {
            d[0] = g[i][0] + 2.f * P.w_sq * x.x;
            d[1] = g[i][1] + 2.f * P.w_sq * x.y;
            d[2] = g[i][2] + 2.f * P.w_sq * x.z;
        } else {
            atomicAdd(d, 2.f * P.w_sq * x.x);
            atomicAdd(d + 1, 2.f * P.w_sq * x.y);
            atomicAdd(d + 2, 2.f * P.w_sq * x.z);
        }
    }
    if (lane == 0) {  // the node's terms; summed in a fixed order by k_loss_reduce
        nt[0] = area;
        nt[1] = vol;
        nt[2] = sq;
    }
}

// per-node terms -> terms, in an order that does not depend on scheduling:
// block b sums the nodes of its contiguous slice (thread t takes every
// kBlock-th node of the slice in turn, then a fixed tree) into partial b;
// one block then adds the kLossParts partials by the same fixed tree.
constexpr int kLossParts = 256;

__device__ inline void block_tree3(double a, double b, double c, double *out)
{
    __shared__ double s[3][kBlock];
    const int t = threadIdx.x;
    s[0][t] = a;
    s[1][t] = b;
    s[2][t] = c;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (t < h) {
            s[0][t] += s[0][t + h];
            s[1][t] += s[1][t + h];
            s[2][t] += s[2][t + h];
        }
        __syncthreads();
    }
    if (t < 3) out[t] = s[t][0];
}

__global__ void __launch_bounds__(256) k_loss_partial(int64_t N, const double *node_terms, double *partial)
{
    const int64_t slice = (N + kLossParts - 1) / kLossParts;
    const int64_t n0 = (int64_t)blockIdx.x * slice, n1 = n0 + slice < N ? n0 + slice : N;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t n = n0 + threadIdx.x; n < n1; n += kBlock) {
        a += node_terms[3 * n];
        b += node_terms[3 * n + 1];
        c += node_terms[3 * n + 2];
    }
    block_tree3(a, b, c, partial + 3 * blockIdx.x);
}

__global__ void __launch_bounds__(256) k_loss_reduce(const double *partial, double *terms)
{
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = t; i < kLossParts; i += kBlock) {
        a += partial[3 * i];
        b += partial[3 * i + 1];
        c += partial[3 * i + 2];
    }
    block_tree3(a, b, c, terms);
}

__global__ void k_zero_f(float *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

__global__ void k_zero_d(double *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// per-node adjoint

struct BParams {
    Inputs in;
    Work w;
    const float *dldx;  // [M][3]
    float *grad_xyz;    // [N][3]
    float *grad_r;      // [N]
};

// The adjoint's per-node scratch in LDS, for nodes of up to VM struts, AC
// arcs and VC vertices.
template <int VM, int AC, int VC>
struct BwdLds {
    SL<float> S[VM + 1];
    float lam_v[VC][3];
    float lam_arc[AC][11];  // o, a, b, t1, t2
    float lam_g[VM + 1][3], lam_h[VM + 1], lam_e[VM + 1][3];
    // circle adjoints per strut: sigma, kappa, frame q, frame r
    float lam_sig[VM + 1], lam_kap[VM + 1], lam_qf[VM + 1][3], lam_rf[VM + 1][3];
    float lam_node[4];      // this node's x, y, z, radius
    float own[VM][4];       // strut-table terms of this node's inputs, per strut
    int s_mbase[AC];
};

// the 4 inputs (x, y, z, radius) of node `node` as dual seeds: direction k
__device__ inline void seed(const float4 c4, int k, V3<Dual> &c, Dual &r)
{
    c = v3(Dual(c4.x, k == 0 ? 1.f : 0.f), Dual(c4.y, k == 1 ? 1.f : 0.f), Dual(c4.z, k == 2 ? 1.f : 0.f));
    r = Dual(c4.w, k == 3 ? 1.f : 0.f);
}

__device__ inline float dotf(const float *a, const float *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__device__ inline void crs(const float *a, const float *b, float *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// The adjoint of node n's mesh vertices, by one wave.  Writes the node's own
// input adjoint to grad_node[n] and, for every incident strut, the part that
// belongs to the far node's inputs to grad_he at the strut's half-edge here;
// k_grad_gather adds them up per node in a fixed order (no atomics between
// nodes, so the gradient's bits do not depend on scheduling).
template <int VM, int AC, int VC>
__device__ void backward_node(const BParams &P, BwdLds<VM, AC, VC> &sm, const int64_t n)
{
    auto &S = sm.S;
    auto &lam_v = sm.lam_v;
    auto &lam_arc = sm.lam_arc;
    auto &lam_g = sm.lam_g;
    auto &lam_h = sm.lam_h;
    auto &lam_e = sm.lam_e;
    auto &lam_sig = sm.lam_sig;
    auto &lam_kap = sm.lam_kap;
    auto &lam_qf = sm.lam_qf;
    auto &lam_rf = sm.lam_rf;
    auto &lam_node = sm.lam_node;
    auto &s_mbase = sm.s_mbase;
    const Work &W = P.w;
    const int64_t N = P.in.n_nodes;
    const int lane = threadIdx.x;
    const int64_t rb = W.node_rec[n];
    // the forward pass or the loss skipped writes: no usable mesh (the
    // gather then writes zeros)
    if (W.flags[0] & (DF_CAPACITY | DF_RECCAP)) return;
    if (rb < 0) return;
    const uint32_t *R = W.rec + rb;
    const int V = (int)R[0], E = (int)R[1], NC = (int)R[2], ncirc = (int)R[3];
    const int wsum = (int)R[4];
    const uint32_t *RV = R + kRecHead;
    const uint32_t *RA = RV + 4 * V;
    const uint32_t *RH = RA + kRecArcFields * E;
    const int64_t row = W.row[n];
    const int v = (int)(W.row[n + 1] - row);
    const int64_t moff = W.node_off[(int64_t)NC_MESH * (N + 1) + n];
    const float4 c4 = W.node4[n];
    const float rho = c4.w;
    const V3<float> cen = v3(c4.x, c4.y, c4.z);
    const float *L = P.dldx + 3 * moff;
    auto af = [&](int f, int j) { return __uint_as_float(RA[kRecArcFields * j + f]); };
    auto vpos = [&](int i, float *w) {
        w[0] = __uint_as_float(RV[4 * i + 1]);
        w[1] = __uint_as_float(RV[4 * i + 2]);
        w[2] = __uint_as_float(RV[4 * i + 3]);
    };

    // ---- strut table, cleared adjoints ------------------------------------
    if (lane < v) {
        const int2 he = W.he[row + lane];
        const float4 f4 = W.node4[he.x];
        bool bad;
        SL<float> s = strut_entry(cen, rho, v3(f4.x, f4.y, f4.z), f4.w, (int)((int64_t)he.x > n), bad);
        s.sid = he.y;
        s.far = he.x;
        S[lane + 1] = s;
    }
    for (int i = lane; i <= VM; i += 64) {
        lam_g[i][0] = lam_g[i][1] = lam_g[i][2] = 0.f;
        lam_h[i] = 0.f;
        lam_e[i][0] = lam_e[i][1] = lam_e[i][2] = 0.f;
        lam_sig[i] = lam_kap[i] = 0.f;
        lam_qf[i][0] = lam_qf[i][1] = lam_qf[i][2] = 0.f;
        lam_rf[i][0] = lam_rf[i][1] = lam_rf[i][2] = 0.f;
    }
    if (lane < 4) lam_node[lane] = 0.f;
    for (int j = lane; j < E; j += 64) {
        s_mbase[j] = (int)RA[kRecArcFields * j + 14];
#pragma unroll
        for (int f = 0; f < 11; ++f) lam_arc[j][f] = 0.f;
    }
    for (int i = lane; i < V; i += 64) {
        lam_v[i][0] = L[3 * i];
        lam_v[i][1] = L[3 * i + 1];
        lam_v[i][2] = L[3 * i + 2];
    }
    __syncthreads();

    // absolute positions are c + w: every mesh vertex of the node moves with c
    {
        const int M = (int)R[5];
        float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll 4
        for (int i = lane; i < M; i += 64) {
            sx += L[3 * i];
            sy += L[3 * i + 1];
            sz += L[3 * i + 2];
        }
        for (int o = 32; o > 0; o >>= 1) {
            sx += __shfl_xor(sx, o, 64);
            sy += __shfl_xor(sy, o, 64);
            sz += __shfl_xor(sz, o, 64);
        }
        if (lane == 0) {
            lam_node[0] += sx;
            lam_node[1] += sy;
            lam_node[2] += sz;
        }
    }

    // Eq. 12 point ii of arc j and its derivative along t
    auto arc_point = [&](int j, float t, float *x, float *dx) {
        float s, c;
        sincos_f32(t, &s, &c);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d] = af(d, j) + af(3 + d, j) * s + af(6 + d, j) * c;
            dx[d] = af(3 + d, j) * c - af(6 + d, j) * s;
        }
    };
    // adds weight lam (a 3-vector) on interior point ii of arc j
    auto add_interior = [&](int j, int ii, const float *lam) {
        const int nseg = (int)(RA[kRecArcFields * j + 13] & 0xffffu);
        const float t1 = af(9, j), t2 = t1 + af(10, j);  // the record keeps dt = t2 - t1
        const float f = (float)ii / (float)nseg;
        const float t = t1 + (t2 - t1) * (float)ii / (float)nseg;
        float s, c;
        sincos_f32(t, &s, &c);
        float g = 0.f;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            atomicAdd(&lam_arc[j][d], lam[d]);
            atomicAdd(&lam_arc[j][3 + d], lam[d] * s);
            atomicAdd(&lam_arc[j][6 + d], lam[d] * c);
            g += lam[d] * (af(3 + d, j) * c - af(6 + d, j) * s);
        }
        atomicAdd(&lam_arc[j][9], (1.f - f) * g);
        atomicAdd(&lam_arc[j][10], f * g);
    };

    // ---- interior points ----------------------------------------------------
    // lane j alone writes arc j's adjoint here: sums in registers, one store
    for (int j = lane; j < E; j += 64) {
        const int nseg = (int)(RA[kRecArcFields * j + 13] & 0xffffu);
        const bool fwd = (RA[kRecArcFields * j + 11] >> 17) & 1u;
        const float t1 = af(9, j), t2 = t1 + af(10, j);  // the record keeps dt = t2 - t1
        float ca[3], cb[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ca[d] = af(3 + d, j);
            cb[d] = af(6 + d, j);
        }
        float acc[11];
#pragma unroll
        for (int f = 0; f < 11; ++f) acc[f] = 0.f;
        const int mb = s_mbase[j];
#pragma unroll 2
        for (int ii = 1; ii < nseg; ++ii) {
            const int li = mb + (fwd ? ii - 1 : nseg - 1 - ii);
            const float lam[3] = {L[3 * li], L[3 * li + 1], L[3 * li + 2]};
            const float f = (float)ii / (float)nseg;
            const float t = t1 + (t2 - t1) * (float)ii / (float)nseg;
            float sn, cs;
            sincos_f32(t, &sn, &cs);
            float g = 0.f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                acc[d] += lam[d];
                acc[3 + d] += lam[d] * sn;
                acc[6 + d] += lam[d] * cs;
                g += lam[d] * (ca[d] * cs - cb[d] * sn);
            }
            acc[9] += (1.f - f) * g;
            acc[10] += f * g;
        }
#pragma unroll
        for (int f = 0; f < 11; ++f) lam_arc[j][f] = acc[f];
    }
    __syncthreads();

    // ---- hole centres (Eq. 13) ----------------------------------------------
    for (int c = lane; c < NC; c += 64) {
        const int li = wsum + c;
        const float lh[3] = {L[3 * li], L[3 * li + 1], L[3 * li + 2]};
        // barycentre as in the forward pass
        float b[3] = {0.f, 0.f, 0.f};
        int cnt = 0;
        for (int j = 0; j < ncirc; ++j) {
            if ((int)(RA[kRecArcFields * j + 13] >> 16) != c) continue;
            const int vs = (int)(RA[kRecArcFields * j + 12] & 0xffffu), ve = (int)(RA[kRecArcFields * j + 12] >> 16);
            float ws[3], we[3];
            vpos(vs, ws);
            vpos(ve, we);
            const int nseg = (int)(RA[kRecArcFields * j + 13] & 0xffffu);
            for (int d = 0; d < 3; ++d) b[d] += 0.5f * (ws[d] + we[d]);
            for (int ii = 1; ii < nseg; ++ii) {
                float x[3], dx[3];
                arc_point(j, af(9, j) + af(10, j) * (float)ii / (float)nseg, x, dx);
                for (int d = 0; d < 3; ++d) b[d] += x[d];
            }
            cnt += nseg;
        }
        for (int d = 0; d < 3; ++d) b[d] /= (float)cnt;
        const float bl = sqrtf(dotf(b, b));
        float dir[3];
        float se[3] = {0.f, 0.f, 0.f}, sl = 1.f;
        const bool use_b = bl >= 1e-3f * rho;
        if (use_b) {
            for (int d = 0; d < 3; ++d) dir[d] = b[d] / bl;
        } else {
            for (int m = 1; m <= v; ++m) {
                se[0] += S[m].ex;
                se[1] += S[m].ey;
                se[2] += S[m].ez;
            }
            sl = sqrtf(dotf(se, se));
            for (int d = 0; d < 3; ++d) dir[d] = -se[d] / sl;
        }
        float sgn = 1.f;
        for (int flip = 0; flip < 2; ++flip) {
            float pm = -1e30f;
            for (int m = 1; m <= v; ++m)
                pm = fmaxf(pm, (S[m].gx * dir[0] + S[m].gy * dir[1] + S[m].gz * dir[2]) * rho - S[m].h);
            if (pm <= 0.f) break;
            for (int d = 0; d < 3; ++d) dir[d] = -dir[d];
            sgn = -sgn;
        }
        // apex rho * dir
        atomicAdd(&lam_node[3], dotf(lh, dir));
        float ld[3];
        for (int d = 0; d < 3; ++d) ld[d] = rho * lh[d];
        const float dl = dotf(dir, ld);
        if (use_b) {
            // dir = sgn b / |b|: lam_b = sgn (ld - dir (dir . ld)) / |b|, then 1/cnt per vertex
            float mu[3];
            for (int d = 0; d < 3; ++d) mu[d] = sgn * (ld[d] - dir[d] * dl) / bl / (float)cnt;
            for (int j = 0; j < ncirc; ++j) {
                if ((int)(RA[kRecArcFields * j + 13] >> 16) != c) continue;
                const int vs = (int)(RA[kRecArcFields * j + 12] & 0xffffu), ve = (int)(RA[kRecArcFields * j + 12] >> 16);
                for (int d = 0; d < 3; ++d) {
                    atomicAdd(&lam_v[vs][d], 0.5f * mu[d]);
                    atomicAdd(&lam_v[ve][d], 0.5f * mu[d]);
                }
                const int nseg = (int)(RA[kRecArcFields * j + 13] & 0xffffu);
                for (int ii = 1; ii < nseg; ++ii) add_interior(j, ii, mu);
            }
        } else {
            // dir = -sgn se / |se|
            for (int m = 1; m <= v; ++m)
                for (int d = 0; d < 3; ++d) {
                    const float g = -sgn * (ld[d] - (-sgn * dir[d]) * (-sgn * dl)) / sl;
                    atomicAdd(&lam_e[m][d], g);
                }
        }
    }
    __syncthreads();

    // ---- arc ends: t1, t2 are the parameters of the end vertices ------------
    // (lane j alone writes arc j's adjoint; vertices are shared: atomics)
    for (int j = lane; j < E; j += 64) {
        const uint32_t u0 = RA[kRecArcFields * j + 11];
        const bool full = (u0 >> 16) & 1u;
        const int vs = (int)(RA[kRecArcFields * j + 12] & 0xffffu), ve = (int)(RA[kRecArcFields * j + 12] >> 16);
        if (full) {
            // the start vertex is the conic point at t = 0: o + b
            for (int d = 0; d < 3; ++d) {
                lam_arc[j][d] += lam_v[vs][d];
                lam_arc[j][6 + d] += lam_v[vs][d];
            }
            continue;
        }
        float o[3], a[3], bb[3], acc[9];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            o[d] = af(d, j);
            a[d] = af(3 + d, j);
            bb[d] = af(6 + d, j);
        }
#pragma unroll
        for (int f = 0; f < 9; ++f) acc[f] = 0.f;
        const float aa = dotf(a, a), bb2 = dotf(bb, bb);
#pragma unroll
        for (int end = 0; end < 2; ++end) {
            const float Lt = lam_arc[j][9 + end];
            const int vi = end ? ve : vs;
            float w[3], r[3];
            vpos(vi, w);
            for (int d = 0; d < 3; ++d) r[d] = w[d] - o[d];
            const float u = dotf(r, a) / aa, vv = dotf(r, bb) / bb2, den = u * u + vv * vv;
            const float lu = Lt * vv / den, lv = -Lt * u / den;
            const float ra = dotf(r, a), rbv = dotf(r, bb);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float lw = lu * a[d] / aa + lv * bb[d] / bb2;
                atomicAdd(&lam_v[vi][d], lw);
                acc[d] -= lw;
                // u = (r . a) / (a . a): du/da = r / aa - 2 a (r . a) / aa^2
                acc[3 + d] += lu * (r[d] / aa - 2.f * a[d] * ra / (aa * aa));
                acc[6 + d] += lv * (r[d] / bb2 - 2.f * bb[d] * rbv / (bb2 * bb2));
            }
        }
#pragma unroll
        for (int f = 0; f < 9; ++f) lam_arc[j][f] += acc[f];
    }
    __syncthreads();

    // ---- conics: (o, a, b) back to the strut table ----------------------------
    // Tangency circle (0, q): o = rho sigma e, a = rho kappa q^, b = rho kappa r^.
    for (int j = lane; j < ncirc; j += 64) {
        const int q = (int)((RA[kRecArcFields * j + 11] >> 8) & 0xffu);
        const SL<float> &sq = S[q];
        float Lo[9];
        for (int f = 0; f < 9; ++f) Lo[f] = lam_arc[j][f];
        const float e[3] = {sq.ex, sq.ey, sq.ez}, qf[3] = {sq.qx, sq.qy, sq.qz}, rf[3] = {sq.rx, sq.ry, sq.rz};
        const float lo_e = dotf(Lo, e), la_q = dotf(Lo + 3, qf), lb_r = dotf(Lo + 6, rf);
        atomicAdd(&lam_node[3], sq.sig * lo_e + sq.kap * (la_q + lb_r));
        atomicAdd(&lam_sig[q], rho * lo_e);
        atomicAdd(&lam_kap[q], rho * (la_q + lb_r));
        for (int d = 0; d < 3; ++d) {
            atomicAdd(&lam_e[q][d], rho * sq.sig * Lo[d]);
            atomicAdd(&lam_qf[q][d], rho * sq.kap * Lo[3 + d]);
            atomicAdd(&lam_rf[q][d], rho * sq.kap * Lo[6 + d]);
        }
    }
    // Ellipse (p, q), Eq. 7, in reverse mode, one lane per arc: the steps of
    // the conic's construction (plane p = q, in-plane axis u1, the completed
    // square) are recomputed, then their adjoints taken in reverse order.
    // Inputs: g_p, h_p, g_q, h_q and rho (kappa_p and sigma_p follow from
    // g_p, h_p and rho, so 1 - |in-plane g_p|^2 = (g_p . n)^2 - (h_p / rho)^2).
    for (int j = ncirc + lane; j < E; j += 64) {
        const uint32_t u0 = RA[kRecArcFields * j + 11];
        const int p = (int)(u0 & 0xffu), q = (int)((u0 >> 8) & 0xffu);
        const SL<float> &Sp = S[p], &Sq = S[q];
        const float gp[3] = {Sp.gx, Sp.gy, Sp.gz}, gq[3] = {Sq.gx, Sq.gy, Sq.gz};
        const float hp = Sp.h, hq = Sq.h;
        float nv[3], nh[3];
        for (int d = 0; d < 3; ++d) nv[d] = gp[d] - gq[d];
        const float nn = sqrtf(dotf(nv, nv));
        for (int d = 0; d < 3; ++d) nh[d] = nv[d] * (1.f / nn);
        const float d0 = (hp - hq) / nn;
        const float gpn = dotf(gp, nh);
        const float epn = fabsf(gpn * Sp.kap), as = fabsf(Sp.sig);
        const float om = (epn - as) * (epn + as) / (Sp.kap * Sp.kap);
        if (!(om > 0.f)) continue;  // not an ellipse: the forward pass kept no arc of it
        float gam[3], u1[3], tv[3] = {0.f, 0.f, 0.f};
        for (int d = 0; d < 3; ++d) gam[d] = gp[d] - nh[d] * gpn;
        const float gl = sqrtf(dotf(gam, gam));
        const bool axis_from_g = gl > 1e-4f * sqrtf(dotf(gp, gp));
        float ml = 1.f;
        if (axis_from_g) {
            for (int d = 0; d < 3; ++d) u1[d] = gam[d] / gl;
            const float un = dotf(u1, nh);
            for (int d = 0; d < 3; ++d) u1[d] -= nh[d] * un;
            const float il = 1.f / sqrtf(dotf(u1, u1));
            for (int d = 0; d < 3; ++d) u1[d] *= il;
        } else {
            tv[fabsf(nh[0]) < 0.9f ? 0 : 1] = 1.f;
            crs(nh, tv, u1);
            ml = sqrtf(dotf(u1, u1));
            for (int d = 0; d < 3; ++d) u1[d] /= ml;
        }
        const float k0 = d0 * gpn - hp;
        const float al0 = gl * k0 / om;
        const float R2 = rho * rho - d0 * d0 + k0 * k0 / om;
        const float R = sqrtf(fmaxf(R2, 0.f)), som = sqrtf(om), A = R / som;
        float cv[3];
        crs(u1, nh, cv);
        // o = d0 nh + al0 u1, a = A u1, b = R (u1 x nh)
        float Lo[3], La[3], Lb[3];
        for (int d = 0; d < 3; ++d) {
            Lo[d] = lam_arc[j][d];
            La[d] = lam_arc[j][3 + d];
            Lb[d] = lam_arc[j][6 + d];
        }
        float L_nh[3], L_u1[3], L_c[3], tmp[3];
        for (int d = 0; d < 3; ++d) {
            L_nh[d] = Lo[d] * d0;
            L_u1[d] = Lo[d] * al0 + La[d] * A;
            L_c[d] = Lb[d] * R;
        }
        float L_d0 = dotf(Lo, nh), L_al0 = dotf(Lo, u1), L_A = dotf(La, u1), L_R = dotf(Lb, cv);
        crs(nh, L_c, tmp);
        for (int d = 0; d < 3; ++d) L_u1[d] += tmp[d];
        crs(L_c, u1, tmp);
        for (int d = 0; d < 3; ++d) L_nh[d] += tmp[d];
        // A = R / sqrt(om), R = sqrt(max(R2, 0))
        L_R += L_A / som;
        float L_om = -0.5f * L_A * A / om;
        const float L_R2 = R > 0.f ? 0.5f * L_R / R : 0.f;
        // R2 = rho^2 - d0^2 + k0^2 / om, al0 = gl k0 / om, k0 = d0 gpn - hp
        float L_rho = 2.f * rho * L_R2;
        L_d0 -= 2.f * d0 * L_R2;
        float L_k0 = 2.f * k0 / om * L_R2;
        L_om -= (k0 / om) * (k0 / om) * L_R2;
        const float L_gl = k0 / om * L_al0;
        L_k0 += gl / om * L_al0;
        L_om -= al0 / om * L_al0;
        L_d0 += gpn * L_k0;
        float L_gpn = d0 * L_k0, L_hp = -L_k0;
        // u1: gam / |gam| (the re-projection and renormalisation have zero
        // derivative: u1 stays a unit vector in the plane), else the unit
        // vector along nh x t
        float L_gam[3];
        for (int d = 0; d < 3; ++d) L_gam[d] = gl > 0.f ? gam[d] * (L_gl / gl) : 0.f;
        const float uu = dotf(u1, L_u1);
        if (axis_from_g) {
            for (int d = 0; d < 3; ++d) L_gam[d] += (L_u1[d] - u1[d] * uu) / gl;
        } else {
            float Pm[3];
            for (int d = 0; d < 3; ++d) Pm[d] = (L_u1[d] - u1[d] * uu) / ml;
            crs(tv, Pm, tmp);
            for (int d = 0; d < 3; ++d) L_nh[d] += tmp[d];
        }
        // gam = g_p - nh gpn
        float L_gp[3];
        const float gn = dotf(L_gam, nh);
        for (int d = 0; d < 3; ++d) {
            L_gp[d] = L_gam[d];
            L_nh[d] -= gpn * L_gam[d];
        }
        L_gpn -= gn;
        // om = gpn^2 - (h_p / rho)^2
        L_gpn += 2.f * gpn * L_om;
        L_hp -= 2.f * hp / (rho * rho) * L_om;
        L_rho += 2.f * hp * hp / (rho * rho * rho) * L_om;
        // gpn = g_p . nh
        for (int d = 0; d < 3; ++d) {
            L_gp[d] += nh[d] * L_gpn;
            L_nh[d] += gp[d] * L_gpn;
        }
        // d0 = (h_p - h_q) / |n|, nh = n / |n|, n = g_p - g_q
        L_hp += L_d0 / nn;
        const float L_hq = -L_d0 / nn, L_nn = -d0 / nn * L_d0;
        const float nl = dotf(nh, L_nh);
        for (int d = 0; d < 3; ++d) {
            const float L_n = (L_nh[d] - nh[d] * nl) / nn + nh[d] * L_nn;
            atomicAdd(&lam_g[p][d], L_gp[d] + L_n);
            atomicAdd(&lam_g[q][d], -L_n);
        }
        atomicAdd(&lam_h[p], L_hp);
        atomicAdd(&lam_h[q], L_hq);
        atomicAdd(&lam_node[3], L_rho);
    }
    __syncthreads();

    // ---- vertices: implicit function theorem on the tie equations ------------
    // F1 = (g_p - g_q) . w - (h_p - h_q), F2 = (g_p - g_r) . w - (h_p - h_r),
    // F3 = g_p . w - h_p - s, F4 = |w|^2 - rho^2 - s^2 (label 0: g = 0, h = 0).
    // J^T mu = (lam_w, 0) gives mu3 = -2 s mu4 and
    // [n1 | n2 | 2 (w - s g_p)] (mu1, mu2, mu4) = lam_w.
    for (int i = lane; i < V; i += 64) {
        const uint32_t name = RV[4 * i];
        const int p = (int)(name >> 24), q = (int)((name >> 16) & 0xffu), r = (int)((name >> 8) & 0xffu);
        if (r == 0xff) continue;  // start point of a whole conic (handled with its arc)
        float w[3], gp[3] = {0.f, 0.f, 0.f}, gq[3], gr[3];
        vpos(i, w);
        float hp = 0.f;
        if (p) {
            gp[0] = S[p].gx; gp[1] = S[p].gy; gp[2] = S[p].gz;
            hp = S[p].h;
        }
        gq[0] = S[q].gx; gq[1] = S[q].gy; gq[2] = S[q].gz;
        gr[0] = S[r].gx; gr[1] = S[r].gy; gr[2] = S[r].gz;
        const float s = dotf(gp, w) - hp;
        float n1[3], n2[3], n3[3];
        for (int d = 0; d < 3; ++d) {
            n1[d] = gp[d] - gq[d];
            n2[d] = gp[d] - gr[d];
            n3[d] = 2.f * (w[d] - s * gp[d]);
        }
        const float lw[3] = {lam_v[i][0], lam_v[i][1], lam_v[i][2]};
        // Cramer on columns n1, n2, n3
        auto det3 = [](const float *a, const float *b, const float *c) {
            return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                   a[2] * (b[0] * c[1] - b[1] * c[0]);
        };
        // solve [n1 n2 n3] x = lw, with the matrix holding n1, n2, n3 as columns
        float m1[3], m2[3], m3[3];
        const float dt = det3(n1, n2, n3);  // det of rows n1, n2, n3 = det of columns
        // x_k = det(matrix with column k replaced by lw) / det
        // (the determinant of a matrix equals that of its transpose)
        for (int d = 0; d < 3; ++d) {
            m1[d] = n1[d];
            m2[d] = n2[d];
            m3[d] = n3[d];
        }
        const float mu1 = det3(lw, m2, m3) / dt;
        const float mu2 = det3(m1, lw, m3) / dt;
        const float mu4 = det3(m1, m2, lw) / dt;
        const float mu3 = -2.f * s * mu4;
        // dL/dtheta = -mu^T dF/dtheta
        const float cp = mu1 + mu2 + mu3;
        if (p) {
            for (int d = 0; d < 3; ++d) atomicAdd(&lam_g[p][d], -cp * w[d]);
            atomicAdd(&lam_h[p], cp);
        }
        for (int d = 0; d < 3; ++d) {
            atomicAdd(&lam_g[q][d], mu1 * w[d]);
            atomicAdd(&lam_g[r][d], mu2 * w[d]);
        }
        atomicAdd(&lam_h[q], -mu1);
        atomicAdd(&lam_h[r], -mu2);
        atomicAdd(&lam_node[3], 2.f * rho * mu4);
    }
    __syncthreads();

    // ---- strut table: g, h, e, sigma, kappa, frame from the two nodes' inputs
    // forward mode, lanes over (strut, input) pairs: 4 inputs of this node,
    // 4 of the far node
    for (int x = lane; x < v * 8; x += 64) {
        const int m = x / 8 + 1, dir = x % 8;
        const int far = S[m].far;
        const float4 f4 = W.node4[far];
        V3<Dual> cd = v3(Dual(c4.x), Dual(c4.y), Dual(c4.z)), cf = v3(Dual(f4.x), Dual(f4.y), Dual(f4.z));
        Dual rd = Dual(c4.w), rf = Dual(f4.w);
        if (dir < 4) seed(c4, dir, cd, rd);
        else seed(f4, dir - 4, cf, rf);
        bool bad;
        const SL<Dual> s = strut_entry(cd, rd, cf, rf, S[m].lower, bad);
        const float g = lam_g[m][0] * s.gx.d + lam_g[m][1] * s.gy.d + lam_g[m][2] * s.gz.d + lam_h[m] * s.h.d +
                        lam_e[m][0] * s.ex.d + lam_e[m][1] * s.ey.d + lam_e[m][2] * s.ez.d + lam_sig[m] * s.sig.d +
                        lam_kap[m] * s.kap.d + lam_qf[m][0] * s.qx.d + lam_qf[m][1] * s.qy.d +
                        lam_qf[m][2] * s.qz.d + lam_rf[m][0] * s.rx.d + lam_rf[m][1] * s.ry.d + lam_rf[m][2] * s.rz.d;
        if (dir < 4) sm.own[m - 1][dir] = g;
        else W.grad_he[4 * (row + m - 1) + dir - 4] = g;
    }
    __syncthreads();
    if (lane < 4) {
        float acc = lam_node[lane];
        for (int m = 0; m < v; ++m) acc += sm.own[m][lane];
        W.grad_node[4 * n + lane] = acc;
    }
}

// nodes of up to kVmax struts, one block (wave) each
__global__ void __launch_bounds__(64) k_backward(BParams P)
{
    __shared__ BwdLds<kVmax, kAcap, kVcap> sm;
    const int64_t n = blockIdx.x;
    if (n >= P.in.n_nodes) return;
    if (P.w.row[n + 1] - P.w.row[n] > kVmax) return;  // k_backward_big
    backward_node(P, sm, n);
}

// nodes of the multi-wave class (queue class 3), one wave each with the
// larger capacities, a fixed grid looping over the class
__global__ void __launch_bounds__(64) k_backward_big(BParams P)
{
    __shared__ BwdLds<kVmaxBig, kAcapBig, kVcapBig> sm;
    const int64_t cnt = P.w.cls_info[3], base = P.w.cls_info[4 + 3];
    for (int64_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        backward_node(P, sm, P.w.queue[base + i]);
        __syncthreads();
    }
}

// gradient of node n = its own part + the parts its neighbours wrote for
// it at the other half-edge of each incident strut, in adjacency order
__global__ void k_grad_gather(BParams P)
{
    const Work &W = P.w;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= P.in.n_nodes) return;
    float g[4] = {0.f, 0.f, 0.f, 0.f};
    if (W.flags[0] & (DF_CAPACITY | DF_RECCAP)) {
        P.grad_xyz[3 * n] = P.grad_xyz[3 * n + 1] = P.grad_xyz[3 * n + 2] = 0.f;
        P.grad_r[n] = 0.f;
        return;
    }
    if (W.node_rec[n] >= 0)
        for (int d = 0; d < 4; ++d) g[d] = W.grad_node[4 * n + d];
    for (int64_t h = W.row[n]; h < W.row[n + 1]; ++h) {
        const int2 he = W.he[h];
        if (W.node_rec[he.x] < 0) continue;
        const int64_t h0 = W.strut_he[2 * (int64_t)he.y], h1 = W.strut_he[2 * (int64_t)he.y + 1];
        const int64_t tw = h0 == h ? h1 : h0;
        for (int d = 0; d < 4; ++d) g[d] += W.grad_he[4 * tw + d];
    }
    P.grad_xyz[3 * n] = g[0];
    P.grad_xyz[3 * n + 1] = g[1];
    P.grad_xyz[3 * n + 2] = g[2];
    P.grad_r[n] = g[3];
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
constexpr int64_t kBigGridBwd = 1024;  // blocks of k_backward_big

}  // namespace

hipError_t launch_loss(const Inputs &in, const Work &w, const FillOut &o, float3 p0, float w_area, float w_vol,
                       float w_sq, float *dldx, double *terms, hipStream_t st)
{
    if (in.n_nodes == 0) {
        k_zero_d<<<1, 64, 0, st>>>(terms, 3);
        return hipGetLastError();
    }
    // nodes whose vertices do not fit the LDS add with atomics: start from 0
    if (o.cap_mesh > 0) k_zero_f<<<grid_for(3 * o.cap_mesh), kBlock, 0, st>>>(dldx, 3 * o.cap_mesh);
    LParams P;
    P.in = in;
    P.w = w;
    P.tri = o.tri;
    P.xyz = o.mesh_xyz;
    P.cap_mesh = o.cap_mesh;
    P.cap_tri = o.cap_tri;
    P.p0 = p0;
    P.w_area = w_area;
    P.w_vol = w_vol;
    P.w_sq = w_sq;
    P.dldx = dldx;
    P.terms = terms;
    k_loss_node<<<(unsigned)in.n_nodes, 64, 0, st>>>(P);
    double *partial = w.loss_node + 3 * (in.n_nodes + 1);  // kLossParts x 3 after the node terms
    k_loss_partial<<<kLossParts, kBlock, 0, st>>>(in.n_nodes, w.loss_node, partial);
    k_loss_reduce<<<1, kBlock, 0, st>>>(partial, terms);
    return hipGetLastError();
}

hipError_t launch_backward(const Inputs &in, const Work &w, const float *dldx, float *grad_xyz, float *grad_r,
                           hipStream_t st)
{
    const int64_t N = in.n_nodes;
    if (N == 0) return hipSuccess;
    BParams P;
    P.in = in;
    P.w = w;
    P.dldx = dldx;
    P.grad_xyz = grad_xyz;
    P.grad_r = grad_r;
    k_backward<<<(unsigned)N, 64, 0, st>>>(P);
    k_backward_big<<<(unsigned)(N < kBigGridBwd ? N : kBigGridBwd), 64, 0, st>>>(P);
    k_grad_gather<<<grid_for(N), kBlock, 0, st>>>(P);
    return hipGetLastError();
}

}  // namespace lm
