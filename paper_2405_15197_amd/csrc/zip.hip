// Strut bands (Sec. 5: a strut is triangulated by connecting the vertices of
// its two arc loops) and the device-side totals.
//
// Each strut end loop arrives as a list of (mesh vertex, phi) in loop order,
// phi increasing cyclically about the strut axis.  The band is the phi-merge
// zipper: with the samples of both loops sorted by (phi, end), the loop at
// the lower node id first on ties, every loop edge u -> u' forms a triangle
// with the last sample of the other loop that precedes u' (cyclically).
// Triangles of loop-A edges come first (in loop order), then those of loop-B
// edges, all oriented outward.
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

__global__ void k_zip(int64_t S, const int64_t *strut_he, const int64_t *he_off, const int32_t *he_len,
                      const int32_t *band_cnt, const int64_t *band_off, const int2 *loop, int32_t *tri,
                      const int32_t *flags)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S || band_cnt[s] == 0) return;
    if (flags[0] & (DF_CAPACITY | DF_BADLAT | DF_LOOPCAP)) return;
    const int64_t ha = strut_he[2 * s], hb = strut_he[2 * s + 1];
    const int2 *A = loop + he_off[ha];
    const int2 *B = loop + he_off[hb];
    const int na = he_len[ha], nb = he_len[hb];
    if (na <= 0 || nb <= 0) return;
    int32_t *T = tri + 3 * band_off[s];
    // rotate each loop to its smallest phi
    int ia0 = 0, ib0 = 0;
    float pa0 = __int_as_float(A[0].y), pb0 = __int_as_float(B[0].y);
    for (int i = 1; i < na; ++i) {
        float p = __int_as_float(A[i].y);
        if (p < pa0) { pa0 = p; ia0 = i; }
    }
    for (int i = 1; i < nb; ++i) {
        float p = __int_as_float(B[i].y);
        if (p < pb0) { pb0 = p; ib0 = i; }
    }
    // before the first sample of the merge, the last samples are the maxima
    int lastA = ia0 == 0 ? na - 1 : ia0 - 1;
    int lastB = ib0 == 0 ? nb - 1 : ib0 - 1;
    int i = 0, j = 0;
    int pa = ia0, pb = ib0;
    while (i < na || j < nb) {
        bool takeA;
        if (j >= nb) takeA = true;
        else if (i >= na) takeA = false;
        else takeA = __int_as_float(A[pa].y) <= __int_as_float(B[pb].y);
        if (takeA) {
            int e = pa == 0 ? na - 1 : pa - 1;  // edge A[e] -> A[pa]
            int32_t *t = T + 3 * e;
            t[0] = A[e].x;
            t[1] = A[pa].x;
            t[2] = B[lastB].x;
            lastA = pa;
            pa = pa + 1 == na ? 0 : pa + 1;
            ++i;
        } else {
            int e = pb == 0 ? nb - 1 : pb - 1;  // edge B[e] -> B[pb]
            int32_t *t = T + 3 * (na + e);
            t[0] = B[pb].x;
            t[1] = B[e].x;
            t[2] = A[lastA].x;
            lastB = pb;
            pb = pb + 1 == nb ? 0 : pb + 1;
            ++j;
        }
    }
}

// Totals (device) and capacity checks for the fill pass.
__global__ void k_totals(int64_t N, int64_t S, const int64_t *node_off, const int64_t *he_off,
                         const int64_t *band_off, int64_t loop_cap, FillOut o, int check, int64_t *totals,
                         int32_t *flags)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t Np1 = N + 1;
    int64_t nv = node_off[0 * Np1 + N], na = node_off[1 * Np1 + N], nh = node_off[2 * Np1 + N];
    int64_t nm = node_off[3 * Np1 + N], nf = node_off[4 * Np1 + N];
    int64_t nb = band_off[S], nl = he_off[2 * S];
    totals[0] = nv;
    totals[1] = na;
    totals[2] = nh;
    totals[3] = nm;
    totals[4] = nb + nf;
    totals[5] = nb;
    totals[6] = nf;
    totals[7] = nl;
    totals[10] = flags[2];
    if (nl > loop_cap) atomicOr(flags, DF_LOOPCAP);
    if (nm > 0x7fffffffLL) atomicOr(flags, DF_LOOPCAP);
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

hipError_t launch_zip(const Inputs &in, const Work &w, const FillOut &o, hipStream_t st)
{
    const int64_t S = in.n_struts;
    if (S > 0)
        k_zip<<<grid_for(S), kBlock, 0, st>>>(S, w.strut_he, w.he_off, w.he_len, w.band_cnt, w.band_off, w.loop,
                                              o.tri, w.flags);
    return hipGetLastError();
}

hipError_t launch_totals(const Inputs &in, const Work &w, const FillOut *o, hipStream_t st)
{
    FillOut oo = o ? *o : FillOut{};
    k_totals<<<1, 64, 0, st>>>(in.n_nodes, in.n_struts, w.node_off, w.he_off, w.band_off, w.loop_cap, oo,
                               o ? 1 : 0, w.totals, w.flags);
    return hipGetLastError();
}

}  // namespace lm
