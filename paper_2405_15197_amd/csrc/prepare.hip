// Lattice preparation (validation and node adjacency) and the device-wide
// exclusive scans used for every offset array.
#include "common.h"

namespace lm {
namespace {

constexpr int kBlock = 256;
constexpr int kSortReg = 16;  // rows up to this length are sorted in registers

__global__ void k_pack(Inputs in, float4 *node4, int32_t *deg)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= in.n_nodes) return;
    node4[i] = make_float4(in.x[i], in.y[i], in.z[i], in.r[i]);
    deg[i] = 0;
}

// Runs of equal keys among neighbouring lanes of a wave (struts listed cell
// by cell share endpoints with their neighbours): the first lane of a run
// does one atomic for the whole run.  Keys of lanes without work must differ
// from every node id (negative, unique per lane).
struct Run {
    int leader, rank, len;
};
__device__ inline Run wave_run(int32_t key)
{
    const int lane = threadIdx.x & 63;
    const int32_t prev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || key != prev;
    const unsigned long long hm = __ballot(head);
    const unsigned long long upto = (2ull << lane) - 1;  // lanes 0..lane (all for lane 63)
    const int leader = 63 - __clzll(hm & upto);
    const unsigned long long above = hm & ~upto;
    const int next = above ? __ffsll(above) - 1 : 64;
    return Run{leader, lane - leader, next - leader};
}

// the two endpoint keys of strut s for the run aggregation (negative: none)
__device__ inline void strut_keys(const Inputs &in, int64_t s, int32_t &ka, int32_t &kb, bool &bad)
{
    const int lane = threadIdx.x & 63;
    ka = -1 - lane;
    kb = -1 - lane;
    bad = false;
    if (s >= in.n_struts) return;
    const int32_t a = in.sa[s], b = in.sb[s];
    if (a < 0 || b < 0 || (int64_t)a >= in.n_nodes || (int64_t)b >= in.n_nodes) {
        bad = true;
        return;
    }
    ka = a;
    if (b != a) kb = b;
}

// Degree histogram; out-of-range endpoints raise DF_BADLAT.
__global__ void k_degree(Inputs in, int32_t *deg, int32_t *flags)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t ka, kb;
    bool bad;
    strut_keys(in, s, ka, kb, bad);
    if (bad) atomicOr(&flags[1], DF_BADLAT);
    const Run ra = wave_run(ka), rb = wave_run(kb);
    if (ka >= 0 && ra.rank == 0) atomicAdd(&deg[ka], ra.len);
    if (kb >= 0 && rb.rank == 0) atomicAdd(&deg[kb], rb.len);
}

__global__ void k_zero(int32_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_scatter(Inputs in, const int64_t *row, int32_t *cursor, int2 *he)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t ka, kb;
    bool bad;
    strut_keys(in, s, ka, kb, bad);
    const Run ra = wave_run(ka), rb = wave_run(kb);
    int32_t ba = 0, bb = 0;
    if (ka >= 0 && ra.rank == 0) ba = atomicAdd(&cursor[ka], ra.len);
    if (kb >= 0 && rb.rank == 0) bb = atomicAdd(&cursor[kb], rb.len);
    ba = __shfl(ba, ra.leader, 64);
    bb = __shfl(bb, rb.leader, 64);
    // the order inside a row is arbitrary here; k_sort_rows fixes it
    if (ka >= 0) he[row[ka] + ba + ra.rank] = make_int2(kb >= 0 ? kb : ka, (int32_t)s);
    if (kb >= 0) he[row[kb] + bb + rb.rank] = make_int2(ka, (int32_t)s);
}

// Incident struts of each node in increasing strut id (canonical labels
// 1..v), then the half-edge index of every strut at its lower and higher
// node id.
__global__ void k_sort_rows(int64_t n_nodes, const int64_t *row, int2 *he, int64_t *strut_he, const int32_t *sa,
                            const int32_t *sb)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    int64_t b = row[n], e = row[n + 1];
    if (e - b <= kSortReg) {
        // in registers: bitonic network over kSortReg slots, empty slots last
        const int v = (int)(e - b);
        int2 x[kSortReg];
#pragma unroll
        for (int i = 0; i < kSortReg; ++i) x[i] = i < v ? he[b + i] : make_int2(0, 0x7fffffff);
#pragma unroll
        for (int k = 2; k <= kSortReg; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
                for (int i = 0; i < kSortReg; ++i) {
                    const int l = i ^ j;
                    if (l > i) {
                        const bool up = (i & k) == 0;
                        const bool sw = up ? x[i].y > x[l].y : x[i].y < x[l].y;
                        const int2 lo = sw ? x[l] : x[i], hi = sw ? x[i] : x[l];
                        x[i] = lo;
                        x[l] = hi;
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kSortReg; ++i)
            if (i < v) he[b + i] = x[i];
        // half-edge ids per strut end, all endpoint loads issued at once
        int32_t lo[kSortReg];
#pragma unroll
        for (int i = 0; i < kSortReg; ++i) {
            lo[i] = 0;
            if (i < v) {
                const int32_t a = sa[x[i].y], c = sb[x[i].y];
                lo[i] = a == c ? -1 : (a < c ? a : c);
            }
        }
#pragma unroll
        for (int i = 0; i < kSortReg; ++i) {
            if (i < v) {
                const int64_t s2 = 2 * (int64_t)x[i].y;
                if (lo[i] < 0) {
                    strut_he[s2] = b + i;
                    strut_he[s2 + 1] = b + i;
                } else {
                    strut_he[s2 + (n == lo[i] ? 0 : 1)] = b + i;
                }
            }
        }
        return;
    } else {
        for (int64_t i = b + 1; i < e; ++i) {
            int2 x = he[i];
            int64_t j = i - 1;
            while (j >= b && he[j].y > x.y) {
                he[j + 1] = he[j];
                --j;
            }
            he[j + 1] = x;
        }
    }
    for (int64_t i = b; i < e; ++i) {
        int32_t s = he[i].y;
        int32_t a = sa[s], c = sb[s];
        int32_t lo = a < c ? a : c;
        if (a == c) {
            strut_he[2 * (int64_t)s] = i;
            strut_he[2 * (int64_t)s + 1] = i;
        } else {
            strut_he[2 * (int64_t)s + (n == lo ? 0 : 1)] = i;
        }
    }
}

// ---------------------------------------------------------------------------
// Multi-column exclusive scan, int32 -> int64: reduce, scan partials, scan
// tiles.  Column c of the source starts at src + c*src_stride, of the
// destination at dst + c*dst_stride; dst[c][n] receives the column total.

constexpr int kScanItems = 8;
constexpr int kTile = kBlock * kScanItems;

__device__ inline int64_t wave_incl_scan(int64_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread across the block; returns the
// exclusive prefix and writes the block total to *total.
__device__ inline int64_t block_excl_scan(int64_t x, int64_t *total)
{
    __shared__ int64_t wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(x);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int64_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + inc - x;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const int32_t *src, int64_t n, int64_t src_stride, int64_t *part,
                                                        int64_t nb)
{
    const int32_t *s = src + blockIdx.y * src_stride;
    int64_t base = (int64_t)blockIdx.x * kTile;
    int64_t acc = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        if (i < n) acc += s[i];
    }
    int64_t tot;
    block_excl_scan(acc, &tot);
    if (threadIdx.x == 0) part[blockIdx.y * nb + blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_scan_partials(int64_t *part, int64_t nb, int64_t *dst, int64_t n,
                                                          int64_t dst_stride)
{
    int64_t *p = part + blockIdx.y * nb;
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
        int64_t i = b0 + threadIdx.x;
        int64_t x = i < nb ? p[i] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan(x, &tot);
        if (i < nb) p[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) dst[blockIdx.y * dst_stride + n] = carry;
}

__global__ void __launch_bounds__(kBlock) k_scan_tiles(const int32_t *src, int64_t n, int64_t src_stride,
                                                       const int64_t *part, int64_t nb, int64_t *dst,
                                                       int64_t dst_stride)
{
    const int32_t *s = src + blockIdx.y * src_stride;
    int64_t *d = dst + blockIdx.y * dst_stride;
    int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int64_t acc = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        v[j] = i < n ? s[i] : 0;
        acc += v[j];
    }
    int64_t tot;
    int64_t ex = block_excl_scan(acc, &tot) + part[blockIdx.y * nb + blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        if (i < n) d[i] = ex;
        ex += v[j];
    }
}

// Valence buckets: one 0/1 column per class, scanned, then node ids are
// placed class by class (in node order within a class).
__global__ void k_class_flags(int64_t N, const int64_t *row, int32_t *flags)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int c = valence_class(row[n + 1] - row[n]);
#pragma unroll
    for (int k = 0; k < kClasses; ++k) flags[k * N + n] = k == c;
}

__global__ void k_class_scatter(int64_t N, const int64_t *row, const int64_t *off, int32_t *queue,
                                int64_t *cls_info)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t Np1 = N + 1;
    int64_t base[kClasses];
    int64_t b = 0;
#pragma unroll
    for (int k = 0; k < kClasses; ++k) {
        base[k] = b;
        b += off[k * Np1 + N];
    }
    if (n == 0) {
#pragma unroll
        for (int k = 0; k < kClasses; ++k) {
            cls_info[k] = off[k * Np1 + N];
            cls_info[4 + k] = base[k];
        }
    }
    if (n >= N) return;
    const int c = valence_class(row[n + 1] - row[n]);
    queue[base[c] + off[c * Np1 + n]] = (int32_t)n;
}

// Node radius from per-strut end radii (Sec. 4.1: a strut is tangent to the
// nodal spheres of its ends, so the end radii at a node agree): the mean of
// the end radii of the node's struts in adjacency (strut id) order; a node
// whose end radii spread by more than rel_tol times that mean is counted.
__global__ void k_end_radii(int64_t N, const int64_t *row, const int2 *he, const int32_t *sa, const float *end_r,
                            float rel_tol, float *radius, int32_t *mismatch)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int64_t h0 = row[n], h1 = row[n + 1];
    float sum = 0.f, lo = 3.0e38f, hi = -3.0e38f;
    for (int64_t h = h0; h < h1; ++h) {
        const int64_t st = he[h].y;
        const float r = end_r[2 * st + (sa[st] == (int32_t)n ? 0 : 1)];
        sum += r;
        lo = fminf(lo, r);
        hi = fmaxf(hi, r);
    }
    // equal end radii give exactly that radius
    const float mean = h1 > h0 ? (hi == lo ? lo : sum / (float)(h1 - h0)) : 0.f;
    radius[n] = mean;
    if (h1 > h0 && hi - lo > rel_tol * fabsf(mean)) atomicAdd(mismatch, 1);
}

// d mean / d end radius = 1 / (struts at the node)
__global__ void k_end_grad(int64_t S, const int64_t *row, const int32_t *sa, const int32_t *sb, const float *grad_r,
                           float *grad_end)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * S) return;
    const int64_t st = i >> 1;
    const int32_t n = (i & 1) ? sb[st] : sa[st];
    const int64_t deg = row[n + 1] - row[n];
    grad_end[i] = deg > 0 ? grad_r[n] / (float)deg : 0.f;
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_end_radii(const Inputs &in, const Work &w, const float *end_r, float rel_tol, float *radius,
                            int32_t *mismatch, hipStream_t st)
{
    if (in.n_nodes > 0)
        k_end_radii<<<grid_for(in.n_nodes, kBlock), kBlock, 0, st>>>(in.n_nodes, w.row, w.he, in.sa, end_r, rel_tol,
                                                                      radius, mismatch);
    return hipGetLastError();
}

hipError_t launch_end_grad(const Inputs &in, const Work &w, const float *grad_r, float *grad_end, hipStream_t st)
{
    if (in.n_struts > 0)
        k_end_grad<<<grid_for(2 * in.n_struts, kBlock), kBlock, 0, st>>>(in.n_struts, w.row, in.sa, in.sb, grad_r,
                                                                         grad_end);
    return hipGetLastError();
}

int64_t scan_tmp_needed(int64_t n, int ncols) { return ((n + kTile - 1) / kTile + 1) * ncols; }

hipError_t launch_scan(const int32_t *src, int64_t *dst, int64_t n, int ncols, int64_t src_stride,
                       int64_t dst_stride, int64_t *tmp, int64_t tmp_len, hipStream_t st)
{
    int64_t nb = (n + kTile - 1) / kTile;
    if (nb < 1) nb = 1;
    if (nb * ncols > tmp_len) return hipErrorInvalidValue;
    dim3 g((unsigned)nb, (unsigned)ncols);
    k_scan_reduce<<<g, kBlock, 0, st>>>(src, n, src_stride, tmp, nb);
    k_scan_partials<<<dim3(1, ncols), kBlock, 0, st>>>(tmp, nb, dst, n, dst_stride);
    k_scan_tiles<<<g, kBlock, 0, st>>>(src, n, src_stride, tmp, nb, dst, dst_stride);
    return hipGetLastError();
}

hipError_t launch_prepare(const Inputs &in, const Work &w, hipStream_t st)
{
    int64_t N = in.n_nodes, S = in.n_struts;
    if (N > 0) k_pack<<<grid_for(N, kBlock), kBlock, 0, st>>>(in, w.node4, w.deg);
    if (S > 0) k_degree<<<grid_for(S, kBlock), kBlock, 0, st>>>(in, w.deg, w.flags);
    hipError_t e = launch_scan(w.deg, w.row, N, 1, 0, 0, w.scan_tmp, w.scan_tmp_len, st);
    if (e != hipSuccess) return e;
    if (N > 0) k_zero<<<grid_for(N, kBlock), kBlock, 0, st>>>(w.deg, N);
    if (S > 0) k_scatter<<<grid_for(S, kBlock), kBlock, 0, st>>>(in, w.row, w.deg, w.he);
    if (N > 0) k_sort_rows<<<grid_for(N, kBlock), kBlock, 0, st>>>(N, w.row, w.he, w.strut_he, in.sa, in.sb);
    // valence buckets (the count columns and offsets are free until the node pass)
    if (N > 0) {
        k_class_flags<<<grid_for(N, kBlock), kBlock, 0, st>>>(N, w.row, w.node_cnt);
        e = launch_scan(w.node_cnt, w.node_off, N, kClasses, N, N + 1, w.scan_tmp, w.scan_tmp_len, st);
        if (e != hipSuccess) return e;
        k_class_scatter<<<grid_for(N, kBlock), kBlock, 0, st>>>(N, w.row, w.node_off, w.queue, w.cls_info);
    }
    return hipGetLastError();
}

}  // namespace lm
