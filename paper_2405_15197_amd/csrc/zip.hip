// Strut bands (Sec. 5: a strut is triangulated by connecting the vertices of
// its two arc loops) and the device-side totals.
//
// Each strut end loop arrives in its node's record as a list of (node-local
// mesh vertex, phi) in loop order, phi increasing cyclically about the strut
// axis.  The band is the phi-merge
// zipper: with the samples of both loops sorted by (phi, end), the loop at
// the lower node id first on ties, every loop edge u -> u' forms a triangle
// with the last sample of the other loop that precedes u' (cyclically).
// Triangles of loop-A edges come first (in loop order), then those of loop-B
// edges, all oriented outward.
#include <type_traits>

#include "common.h"

namespace lm {
namespace {

constexpr int kBlock = 256;

__global__ void k_band_count(int64_t S, const int32_t *sa, const int32_t *sb, const int64_t *strut_he,
                             const int32_t *he_len, const int32_t *node_status, int32_t *band_cnt,
                             int64_t *totals)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    int32_t a = sa[s], b = sb[s];
    int32_t c = 0;
    if (a != b && node_status[a] == 0 && node_status[b] == 0)
        c = he_len[strut_he[2 * s]] + he_len[strut_he[2 * s + 1]];
    else
        atomicAdd((unsigned long long *)&totals[9], 1ull);
    band_cnt[s] = c;
}

__global__ void k_bad_nodes(int64_t N, const int32_t *node_status, int64_t *totals)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N && node_status[n] != 0) atomicAdd((unsigned long long *)&totals[8], 1ull);
}

// One wave per G consecutive struts.  Lanes load the struts' loop
// descriptors, the loops are staged in LDS in sorted (phi) order when they
// fit, then lanes run over the group's band triangles in output order
// (coalesced writes).  The apex of a loop-edge triangle is the cyclic
// predecessor of the edge's end among the other loop's samples in
// (phi, end) order, found by binary search on the sorted samples.  The
// staging buffer is kept at 4 KB so that eight waves fit a SIMD; G shrinks
// with the resolution so that a group's loops still fit it.
constexpr int kZipStage = 512;  // staged samples per wave (4 KB of LDS)

// Loop access in sorted order: from LDS (already rotated) or from the node
// record (rotated on the fly).
struct LoopLds {
    const int2 *p;
    int n;
    __device__ int2 at(int k) const { return p[k]; }
};
struct LoopGlobal {
    const int2 *p;
    int n, rot;
    __device__ int2 at(int k) const
    {
        int i = rot + k;
        return p[i >= n ? i - n : i];
    }
};

// number of samples with phi < x (or <= x) minus one, cyclically: the sorted
// index of the predecessor of x
template <typename L>
__device__ inline int pred_sorted(const L &lp, float x, bool inclusive)
{
    int lo = 0, hi = lp.n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const float p = __int_as_float(lp.at(mid).y);
        if (inclusive ? (p <= x) : (p < x)) lo = mid + 1;
        else hi = mid;
    }
    return lo == 0 ? lp.n - 1 : lo - 1;
}

// Triangle j of a band: j < na are the edges of loop A (lower node id), in
// loop order from A's loop position 0; then the edges of loop B.  Edge
// X[k] -> X[k+1] of loop X takes as apex the last sample of the other loop Y
// before X[k+1]: strictly before for edges of A, at or before for edges of B.
// One path for both kinds (lanes of a wave hold both), the loops chosen per
// lane.
template <typename L>
__device__ inline void band_tri(const L &A, const L &B, int ra, int rb, int j, int32_t ma, int32_t mb, int32_t *T)
{
    const bool ea = j < A.n;
    const L X = ea ? A : B, Y = ea ? B : A;
    int k0 = ea ? j - ra : j - A.n - rb;
    if (k0 < 0) k0 += X.n;
    const int k1 = k0 + 1 == X.n ? 0 : k0 + 1;
    const int2 u = X.at(k0), u2 = X.at(k1);
    const int ap = pred_sorted(Y, __int_as_float(u2.y), !ea);
    const int32_t mx = ea ? ma : mb, my = ea ? mb : ma;
    // outward: A edges run u -> u', B edges u' -> u
    T[0] = mx + (ea ? u.x : u2.x);
    T[1] = mx + (ea ? u2.x : u.x);
    T[2] = my + Y.at(ap).x;
}

template <int G>
__global__ void __launch_bounds__(64) k_zip(int64_t S, const int64_t *band_off, const int64_t *strut_he,
                                            const int64_t *he_loop, const int32_t *he_len, const int32_t *he_rot,
                                            const int2 *loop, const int32_t *sa, const int32_t *sb,
                                            const int64_t *mesh_off, int32_t *tri, const int32_t *flags)
{
    __shared__ int2 st[kZipStage];
    __shared__ int64_t g_la[G], g_lb[G];
    __shared__ int g_na[G], g_nb[G], g_ra[G], g_rb[G];
    __shared__ int g_ma[G], g_mb[G], g_t[G + 1], g_q[G + 1];
    if (flags[0] & (DF_CAPACITY | DF_BADLAT | DF_RECCAP)) return;
    const int lane = threadIdx.x;
    const int64_t s0 = xcd_block(blockIdx.x, gridDim.x) * G;
    if (s0 >= S) return;
    const int ns = S - s0 < G ? (int)(S - s0) : G;
    const int64_t t0 = band_off[s0];
    int cnt = 0, q = 0;
    if (lane < ns) {
        const int64_t s = s0 + lane;
        cnt = (int)(band_off[s + 1] - band_off[s]);
        int na = 0, nb = 0;
        if (cnt > 0) {
            const int64_t ha = strut_he[2 * s], hb = strut_he[2 * s + 1];
            na = he_len[ha];
            nb = he_len[hb];
            g_la[lane] = he_loop[ha];
            g_lb[lane] = he_loop[hb];
            g_ra[lane] = he_rot[ha];
            g_rb[lane] = he_rot[hb];
            const int32_t a = sa[s], b = sb[s];
            g_ma[lane] = (int32_t)mesh_off[a < b ? a : b];
            g_mb[lane] = (int32_t)mesh_off[a < b ? b : a];
        }
        g_na[lane] = na;
        g_nb[lane] = nb;
        q = na + nb;
    }
    // prefix sums of the triangle and sample counts over the group
    int ct = cnt, cq = q;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        const int yt = __shfl_up(ct, d, 64), yq = __shfl_up(cq, d, 64);
        if (lane >= d) {
            ct += yt;
            cq += yq;
        }
    }
    if (lane < ns) {
        g_t[lane + 1] = ct;
        g_q[lane + 1] = cq;
    }
    if (lane == 0) {
        g_t[0] = 0;
        g_q[0] = 0;
    }
    __syncthreads();
    const int ntri = g_t[ns], nsamp = g_q[ns];
    const bool staged = nsamp <= kZipStage;
    if (staged) {
        // samples of strut i: loop A sorted, then loop B sorted
        int i = 0;  // x only grows: the strut index carries over
        for (int x = lane; x < nsamp; x += 64) {
            while (g_q[i + 1] <= x) ++i;
            int k = x - g_q[i];
            const int na = g_na[i];
            int64_t base;
            int n, r;
            if (k < na) {
                base = g_la[i];
                n = na;
                r = g_ra[i];
            } else {
                k -= na;
                base = g_lb[i];
                n = g_nb[i];
                r = g_rb[i];
            }
            int idx = r + k;
            if (idx >= n) idx -= n;
            st[x] = loop[base + idx];
        }
        __syncthreads();
    }
    int i = 0;
    for (int x = lane; x < ntri; x += 64) {
        while (g_t[i + 1] <= x) ++i;
        const int j = x - g_t[i];
        int32_t *T = tri + 3 * (t0 + x);
        if (staged) {
            const LoopLds A{st + g_q[i], g_na[i]}, B{st + g_q[i] + g_na[i], g_nb[i]};
            band_tri(A, B, g_ra[i], g_rb[i], j, g_ma[i], g_mb[i], T);
        } else {
            const LoopGlobal A{loop + g_la[i], g_na[i], g_ra[i]}, B{loop + g_lb[i], g_nb[i], g_rb[i]};
            band_tri(A, B, g_ra[i], g_rb[i], j, g_ma[i], g_mb[i], T);
        }
    }
}

// Totals (device) and capacity checks for the fill pass.
__global__ void k_totals(int64_t N, int64_t S, const int64_t *node_off, const unsigned long long *rec_top,
                         const int64_t *band_off, FillOut o, int check, int64_t *totals, int32_t *flags)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t Np1 = N + 1;
    int64_t nv = node_off[0 * Np1 + N], na = node_off[1 * Np1 + N], nh = node_off[2 * Np1 + N];
    int64_t nm = node_off[3 * Np1 + N], nf = node_off[4 * Np1 + N];
    int64_t nb = band_off[S];
    unsigned long long top = 0;  // record words: the fullest region times the region count
    for (int g = 0; g < kRecRegions; ++g) top = rec_top[g] > top ? rec_top[g] : top;
    const int64_t nl = (int64_t)top * kRecRegions * 4;
    totals[0] = nv;
    totals[1] = na;
    totals[2] = nh;
    totals[3] = nm;
    totals[4] = nb + nf;
    totals[5] = nb;
    totals[6] = nf;
    totals[7] = nl;
    totals[10] = flags[2];
    if (nm > 0x7fffffffLL) atomicOr(flags, DF_RECCAP);
    if (check) {
        bool bad = nm > o.cap_mesh || nb + nf > o.cap_tri;
        if (o.vert_name && nv > o.cap_vert) bad = true;
        if (o.arc_f32 && na > o.cap_arc) bad = true;
        if (bad) atomicOr(flags, DF_CAPACITY);
    }
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_band_count(const Inputs &in, const Work &w, hipStream_t st)
{
    const int64_t N = in.n_nodes, S = in.n_struts;
    const int32_t *status = w.node_cnt + (int64_t)NC_STATUS * N;
    if (N > 0) k_bad_nodes<<<grid_for(N), kBlock, 0, st>>>(N, status, w.totals);
    if (S > 0)
        k_band_count<<<grid_for(S), kBlock, 0, st>>>(S, in.sa, in.sb, w.strut_he, w.he_len, status, w.band_cnt,
                                                     w.totals);
    return hipGetLastError();
}

hipError_t launch_zip(const Inputs &in, const Work &w, const FillOut &o, int k, hipStream_t st)
{
    const int64_t S = in.n_struts;
    if (S == 0) return hipSuccess;
    // a band has about 2 (k + 4) samples: groups whose loops fill most of
    // the staging buffer
    const int64_t *mo = w.node_off + (int64_t)NC_MESH * (in.n_nodes + 1);
    const int2 *loop = (const int2 *)w.rec;
    auto go = [&](auto g) {
        constexpr int G = decltype(g)::value;
        k_zip<G><<<(unsigned)((S + G - 1) / G), 64, 0, st>>>(S, w.band_off, w.strut_he, w.he_loop, w.he_len,
                                                              w.he_rot, loop, in.sa, in.sb, mo, o.tri, w.flags);
    };
    if (k <= 24) go(std::integral_constant<int, 8>{});
    else if (k <= 32) go(std::integral_constant<int, 6>{});
    else if (k <= 56) go(std::integral_constant<int, 4>{});
    else go(std::integral_constant<int, 2>{});
    return hipGetLastError();
}

hipError_t launch_totals(const Inputs &in, const Work &w, const FillOut *o, hipStream_t st)
{
    FillOut oo = o ? *o : FillOut{};
    k_totals<<<1, 64, 0, st>>>(in.n_nodes, in.n_struts, w.node_off, w.rec_top, w.band_off, oo, o ? 1 : 0,
                               w.totals, w.flags);
    return hipGetLastError();
}

}  // namespace lm
