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

// One thread per band triangle, in output order (coalesced writes).  The
// apex of a loop-edge triangle is the cyclic predecessor of the edge's end
// among the other loop's samples in (phi, end) order, found by binary search
// on that loop read from its smallest phi onwards.
__device__ inline int pred_sorted(const int2 *L, int n, int rot, float x, bool inclusive)
{
    // number of samples with phi < x (or <= x), in sorted order
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int pos = rot + mid;
        if (pos >= n) pos -= n;
        float p = __int_as_float(L[pos].y);
        bool before = inclusive ? (p <= x) : (p < x);
        if (before) lo = mid + 1;
        else hi = mid;
    }
    int i = lo == 0 ? n - 1 : lo - 1;
    int pos = rot + i;
    return pos >= n ? pos - n : pos;
}

__global__ void __launch_bounds__(kBlock) k_zip(int64_t S, const int64_t *band_off, const int64_t *strut_he,
                                                const int64_t *he_loop, const int32_t *he_len, const int32_t *he_rot,
                                                const int2 *loop, const int32_t *sa, const int32_t *sb,
                                                const int64_t *mesh_off, int32_t *tri, const int32_t *flags)
{
    if (flags[0] & (DF_CAPACITY | DF_BADLAT | DF_RECCAP)) return;
    const int64_t nband = band_off[S];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x;  // first triangle of the block
    if (t0 >= nband) return;
    // strut of the block's first triangle, then of this thread's (searching
    // forward from there)
    __shared__ int64_t s_first;
    if (threadIdx.x == 0) {
        int64_t lo = 0, hi = S - 1;  // last s with band_off[s] <= t0
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) >> 1;
            if (band_off[mid] <= t0) lo = mid;
            else hi = mid - 1;
        }
        s_first = lo;
    }
    __syncthreads();
    if (t >= nband) return;
    int64_t lo = s_first, hi = S - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (band_off[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const int64_t s = lo;
    const int j = (int)(t - band_off[s]);
    const int64_t ha = strut_he[2 * s], hb = strut_he[2 * s + 1];
    const int2 *A = loop + he_loop[ha];
    const int2 *B = loop + he_loop[hb];
    const int na = he_len[ha], nb = he_len[hb];
    // loop A is at the lower node id
    const int32_t a = sa[s], b = sb[s];
    const int32_t ma = (int32_t)mesh_off[a < b ? a : b], mb = (int32_t)mesh_off[a < b ? b : a];
    int32_t *T = tri + 3 * t;
    if (j < na) {
        // edge A[j] -> A[j+1]; apex: last B sample strictly before A[j+1]
        int j2 = j + 1 == na ? 0 : j + 1;
        int2 u2 = A[j2];
        int ap = pred_sorted(B, nb, he_rot[hb], __int_as_float(u2.y), false);
        T[0] = ma + A[j].x;
        T[1] = ma + u2.x;
        T[2] = mb + B[ap].x;
    } else {
        // edge B[e] -> B[e+1]; apex: last A sample at or before B[e+1]
        int e = j - na;
        int e2 = e + 1 == nb ? 0 : e + 1;
        int2 w2 = B[e2];
        int ap = pred_sorted(A, na, he_rot[ha], __int_as_float(w2.y), true);
        T[0] = mb + w2.x;
        T[1] = mb + B[e].x;
        T[2] = ma + A[ap].x;
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

hipError_t launch_zip(const Inputs &in, const Work &w, const FillOut &o, hipStream_t st)
{
    const int64_t S = in.n_struts;
    // grid sized for the capacity; blocks past the band total exit at once
    int64_t cap = o.cap_tri;
    if (S > 0 && cap > 0)
        k_zip<<<grid_for(cap), kBlock, 0, st>>>(S, w.band_off, w.strut_he, w.he_loop, w.he_len, w.he_rot,
                                                (const int2 *)w.rec, in.sa, in.sb,
                                                w.node_off + (int64_t)NC_MESH * (in.n_nodes + 1), o.tri, w.flags);
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
