// Sink mode: the lattice is meshed in ranges of node ids (chunks, or groups
// of whole parts) and the triangles are reduced to counts and
// order-independent hashes instead of being stored (for lattices whose mesh
// does not fit in memory).
//
// A range's node list is the range plus its halo: every neighbour with a
// higher id outside the range (the band of a strut is emitted by the range of
// its lower end, which needs the other end's loop).  The node pass in sink
// mode hashes the vertices and fans of the range's own nodes and keeps only
// the strut end loops; the kernels here list the range's struts and hash
// their bands.  Names, keys and words: see the sink section of common.h.
// Ranges are processed back to back on the stream without host
// synchronisation: sizes are read on the device, and a range whose records
// did not fit is marked for a second run.
#include "common.h"

namespace lm {
namespace {

constexpr int kSlots = kSinkSlots;
constexpr int kWords = kSinkWords;

// Wave-aggregated append of `value` to list `k` (when active): one atomic
// per list and wave.  All lanes of the wave must call it.
__device__ inline void append(bool active, int k, int32_t value, int32_t *lists, int64_t cap, int32_t *cnt)
{
    const int lane = threadIdx.x & 63;
    for (int c = 0; c < kClasses; ++c) {
        const unsigned long long m = __ballot(active && k == c);
        if (m == 0) continue;
        const int leader = __ffsll((long long)m) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&cnt[c], __popcll(m));
        base = __shfl(base, leader, 64);
        if (active && k == c) lists[c * cap + base + __popcll(m & ((1ull << lane) - 1ull))] = value;
    }
}

// The list builders run in blocks of kListBlock threads (four waves).
constexpr int kListBlock = 256;
constexpr int kListWaves = kListBlock / 64;

// Inclusive sum over the wave (lanes below first).
template <typename T>
__device__ inline T wave_incl_sum(T x)
{
    const int lane = threadIdx.x & 63;
    for (int d = 1; d < 64; d <<= 1) {
        const T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive sum of x over the block and the block's total: the waves' own
// sums meet in LDS.  All threads of the block call it, once per kernel (a
// second call could overwrite the wave sums before every wave has read them).
template <typename T>
__device__ inline T block_excl_sum(T x, T &total)
{
    __shared__ T s_w[kListWaves];
    const int wv = threadIdx.x >> 6;
    const T inc = wave_incl_sum(x);
    if ((threadIdx.x & 63) == 63) s_w[wv] = inc;
    __syncthreads();
    T pre = 0, tot = 0;
    for (int w = 0; w < kListWaves; ++w) {
        const T t = s_w[w];
        if (w < wv) pre += t;
        tot += t;
    }
    total = tot;
    return pre + inc - x;
}

// Chunk node list in valence classes: the range (entries reserved per block,
// one atomic per class and block; a thread's class is a 16-bit field of a
// packed count), then the halo (marked with the chunk's epoch so that each
// halo node is listed once; few nodes, appended per wave).
__global__ void __launch_bounds__(kListBlock) k_chunk_list(int64_t n0, int64_t n1, const int64_t *row, const int2 *he,
                                                           int32_t *mark, int32_t epoch, int32_t *lists, int64_t cap,
                                                           int32_t *cnt, int t16, int t32)
{
    static_assert(kClasses * 16 <= 64 && kListBlock < 65536, "class counts are 16-bit fields of one word");
    __shared__ int32_t s_base[kClasses];
    const int64_t n = n0 + (int64_t)blockIdx.x * kListBlock + threadIdx.x;
    const bool in = n < n1;
    int64_t r0 = 0, r1 = 0;
    if (in) {
        r0 = row[n];
        r1 = row[n + 1];
    }
    const int cls = in ? valence_class(r1 - r0, t16, t32) : 0;
    const uint64_t one = in ? 1ull << (16 * cls) : 0ull;
    uint64_t tot;
    const uint64_t ex = block_excl_sum(one, tot);
    if (threadIdx.x < kClasses) {
        const int c = (int)((tot >> (16 * threadIdx.x)) & 0xffff);
        s_base[threadIdx.x] = c ? atomicAdd(&cnt[threadIdx.x], c) : 0;
    }
    __syncthreads();
    if (in) lists[cls * cap + s_base[cls] + (int64_t)((ex >> (16 * cls)) & 0xffff)] = (int32_t)n;
    int deg = (int)(r1 - r0);
    int maxdeg = deg;
    for (int o = 32; o > 0; o >>= 1) maxdeg = max(maxdeg, __shfl_xor(maxdeg, o, 64));
    for (int i = 0; i < maxdeg; ++i) {
        bool add = false;
        int32_t far = 0;
        int k = 0;
        if (i < deg) {
            far = he[r0 + i].x;
            if ((int64_t)far > n && (int64_t)far >= n1) {
                add = atomicExch(&mark[far], epoch) != epoch;
                if (add) k = valence_class(row[far + 1] - row[far], t16, t32);
            }
        }
        append(add, k, far, lists, cap, cnt);
    }
}

__global__ void k_chunk_info(const int32_t *cnt, int64_t cap, int64_t *info)
{
    if (threadIdx.x < kClasses) {
        info[threadIdx.x] = cnt[threadIdx.x];
        info[4 + threadIdx.x] = (int64_t)threadIdx.x * cap;
    }
}

// Struts whose lower end is in the range and whose ends both have a mesh:
// each thread counts its node's, the block reserves its entries with one
// atomic, and the thread writes them (the first 64 half-edges' verdicts are
// kept as a mask, later ones tested again).
__global__ void __launch_bounds__(kListBlock) k_chunk_struts(int64_t n0, int64_t n1, const int64_t *row,
                                                             const int2 *he, const int64_t *node_rec, int32_t *list,
                                                             int32_t *cnt)
{
    __shared__ int32_t s_base;
    const int64_t n = n0 + (int64_t)blockIdx.x * kListBlock + threadIdx.x;
    int64_t r0 = 0, r1 = 0;
    if (n < n1 && node_rec[n] >= 0) {
        r0 = row[n];
        r1 = row[n + 1];
    }
    auto owned = [&](const int2 h) { return (int64_t)h.x > n && node_rec[h.x] >= 0; };
    int c = 0;
    uint64_t m = 0;
    for (int64_t r = r0; r < r1; ++r)
        if (owned(he[r])) {
            ++c;
            if (r - r0 < 64) m |= 1ull << (r - r0);
        }
    int tot;
    int32_t at = block_excl_sum(c, tot);
    if (threadIdx.x == 0) s_base = tot ? atomicAdd(cnt, tot) : 0;
    __syncthreads();
    at += s_base;
    while (m) {
        list[at++] = he[r0 + __builtin_ctzll(m)].y;
        m &= m - 1;
    }
    for (int64_t r = r0 + 64; r < r1; ++r) {
        const int2 h = he[r];
        if (owned(h)) list[at++] = h.y;
    }
}

// Bands of the listed struts (one wave per G), hashed.  A 4 KB staging
// buffer lets eight waves share a SIMD; G shrinks with the resolution so
// that a group's loops still fit it.
constexpr int kZipStage = 512;
constexpr int64_t kZipGrid = 256 * 64;  // blocks (waves) of a band launch

template <int G>
__global__ void __launch_bounds__(64) k_sink_zip(Work W, SinkOut P, const int32_t *list, const int32_t *cnt,
                                                 const int32_t *sa, const int32_t *sb)
{
    __shared__ int2 st[kZipStage];
    __shared__ int g_na[G], g_nb[G], g_ra[G], g_rb[G];
    __shared__ int64_t g_la[G], g_lb[G], g_a[G], g_b[G];
    __shared__ int g_t[G + 1];
    __shared__ unsigned long long g_h[G];  // triangle-key sum per strut
    const int lane = threadIdx.x;
    const int64_t ns_all = *cnt;
    // a fixed grid walks the range's strut list (its length is on the device)
    for (int64_t g0 = (int64_t)blockIdx.x * G; g0 < ns_all; g0 += (int64_t)gridDim.x * G) {
        const int ns = ns_all - g0 < G ? (int)(ns_all - g0) : G;
        int c = 0;
        if (lane < ns) {
            const int64_t s = list[g0 + lane];
            const int64_t ha = W.strut_he[2 * s], hb = W.strut_he[2 * s + 1];
            g_na[lane] = W.he_len[ha];
            g_nb[lane] = W.he_len[hb];
            g_la[lane] = W.he_loop[ha];
            g_lb[lane] = W.he_loop[hb];
            g_ra[lane] = W.he_rot[ha];
            g_rb[lane] = W.he_rot[hb];
            const int32_t a = sa[s], b = sb[s];
            g_a[lane] = a < b ? a : b;
            g_b[lane] = a < b ? b : a;
            c = g_na[lane] + g_nb[lane];
            g_h[lane] = 0ull;
        }
        int ct = c;
    #pragma unroll
        for (int d = 1; d < G; d <<= 1) {
            const int y = __shfl_up(ct, d, 64);
            if (lane >= d) ct += y;
        }
        if (lane < ns) g_t[lane + 1] = ct;
        if (lane == 0) g_t[0] = 0;
        __syncthreads();
        const int ntri = g_t[ns];
        const bool staged = ntri <= kZipStage;
        const int2 *loops = (const int2 *)W.rec;
        if (staged) {
            int i = 0;  // x only grows: the strut index carries over
            for (int x = lane; x < ntri; x += 64) {
                while (g_t[i + 1] <= x) ++i;
                int k = x - g_t[i];
                int64_t base;
                int n, r;
                if (k < g_na[i]) {
                    base = g_la[i]; n = g_na[i]; r = g_ra[i];
                } else {
                    k -= g_na[i]; base = g_lb[i]; n = g_nb[i]; r = g_rb[i];
                }
                int idx = r + k;
                if (idx >= n) idx -= n;
                st[x] = loops[base + idx];
            }
            __syncthreads();
        }
        int i = 0;
        for (int x = lane; x < ntri; x += 64) {
            uint64_t ht = 0;
            while (g_t[i + 1] <= x) ++i;
            const int j = x - g_t[i];
            const int na = g_na[i], nb = g_nb[i], ra = g_ra[i], rb = g_rb[i];
            // edge j runs along loop X (A for j < na, else B); its apex is
            // the last sample of the other loop Y before the edge's end
            // (strictly before for edges of A, at or before for edges of B).
            // One path for both kinds, the loops chosen per lane.
            const bool ea = j < na;
            const int nx = ea ? na : nb, ny = ea ? nb : na;
            const int rx = ea ? ra : rb, ry = ea ? rb : ra;
            const int ox = ea ? 0 : na, oy = ea ? na : 0;  // staged: A then B
            const int64_t lx = ea ? g_la[i] : g_lb[i], ly = ea ? g_lb[i] : g_la[i];
            // sorted-order views of both loops (LDS when staged)
            auto X = [&](int k) -> int2 {
                if (staged) return st[g_t[i] + ox + k];
                const int q = rx + k;
                return loops[lx + (q >= nx ? q - nx : q)];
            };
            auto Y = [&](int k) -> int2 {
                if (staged) return st[g_t[i] + oy + k];
                const int q = ry + k;
                return loops[ly + (q >= ny ? q - ny : q)];
            };
            int k0 = j - ox - rx;
            if (k0 < 0) k0 += nx;
            const int k1 = k0 + 1 == nx ? 0 : k0 + 1;
            const int2 u = X(k0), u2 = X(k1);
            const float xv = __int_as_float(u2.y);
            int lo = 0, hi = ny;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const float p = __int_as_float(Y(mid).y);
                if (ea ? (p < xv) : (p <= xv)) lo = mid + 1;
                else hi = mid;
            }
            const int ap = lo == 0 ? ny - 1 : lo - 1;
            const int64_t xn = sink_local_node(P, ea ? g_a[i] : g_b[i]), yn = sink_local_node(P, ea ? g_b[i] : g_a[i]);
            // outward: A edges run u -> u', B edges u' -> u
            ht += tri_key(vid_of(xn, ea ? u.x : u2.x), vid_of(xn, ea ? u2.x : u.x), vid_of(yn, Y(ap).x));
            atomicAdd(&g_h[i], (unsigned long long)ht);
        }
        __syncthreads();
        // per part of the struts' lower nodes (runs of equal parts flushed once)
        if (lane == 0) {
            int32_t cur = P.node_part ? P.node_part[g_a[0]] : 0;
            uint64_t cnt_s = 0, h_s = 0;
            for (int i = 0; i < ns; ++i) {
                const int32_t pt = P.node_part ? P.node_part[g_a[i]] : 0;
                if (pt != cur) {
                    sink_add(P, cur, 0, cnt_s);
                    sink_add(P, cur, 1, h_s);
                    cur = pt;
                    cnt_s = h_s = 0;
                }
                cnt_s += (uint64_t)(g_t[i + 1] - g_t[i]);
                h_s += g_h[i];
            }
            sink_add(P, cur, 0, cnt_s);
            sink_add(P, cur, 1, h_s);
        }
        __syncthreads();  // the group's shared arrays are reused
    }
}

// slots -> the chunk's output words; clears the slots
__global__ void k_sink_reduce(unsigned long long *slots, uint64_t *out)
{
    const int w = threadIdx.x;
    if (w >= kWords) return;
    uint64_t s = 0;
    for (int i = 0; i < kSlots; ++i) {
        s += slots[i * kWords + w];
        slots[i * kWords + w] = 0;
    }
    out[w] = s;
}

// A range's node pass is over: keep whether its records overflowed (the
// range is run again) and clear the flag for the next range.
__global__ void k_range_done(int32_t *flags, int32_t *fail, int64_t r)
{
    if (threadIdx.x != 0) return;
    fail[r] = flags[0] & DF_RECCAP;
    flags[0] = 0;
    flags[2] = 0;
}

// zero the per-part slots of parts [p0, p1)
__global__ void k_clear_parts(unsigned long long *slots, int64_t p0, int64_t p1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (p1 - p0) * kSlots * kWords;
    if (i < n) slots[p0 * kSlots * kWords + i] = 0ull;
}

// part (binary search in the part offsets) and resolution of every node
__global__ void k_part_map(int64_t N, const int64_t *part_off, const int32_t *part_k, int64_t n_parts,
                           int32_t *node_part, int16_t *node_k)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    int64_t lo = 0, hi = n_parts - 1;  // last part with part_off <= n
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (part_off[mid] <= n) lo = mid;
        else hi = mid - 1;
    }
    node_part[n] = (int32_t)lo;
    node_k[n] = (int16_t)part_k[lo];
}

// per-part slots -> out[part][kWords]
__global__ void k_parts_reduce(const unsigned long long *slots, int64_t n_parts, uint64_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_parts * kWords) return;
    const int64_t p = i / kWords, w = i % kWords;
    uint64_t s = 0;
    for (int j = 0; j < kSlots; ++j) s += slots[(p * kSlots + j) * kWords + w];
    out[i] = s;
}

inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int64_t sink_slots_words() { return (int64_t)kSlots * kWords; }

hipError_t launch_part_map(int64_t N, const int64_t *part_off, const int32_t *part_k, int64_t n_parts,
                           int32_t *node_part, int16_t *node_k, hipStream_t st)
{
    if (N > 0) k_part_map<<<grid_for(N, 256), 256, 0, st>>>(N, part_off, part_k, n_parts, node_part, node_k);
    return hipGetLastError();
}

hipError_t launch_parts_reduce(const unsigned long long *slots, int64_t n_parts, uint64_t *out, hipStream_t st)
{
    if (n_parts > 0) k_parts_reduce<<<grid_for(n_parts * kWords, 256), 256, 0, st>>>(slots, n_parts, out);
    return hipGetLastError();
}

hipError_t launch_chunk_list(const Work &w, int64_t n0, int64_t n1, int32_t *mark, int32_t epoch, int32_t *lists,
                             int64_t cap, int32_t *cnt, int64_t *info, int t16, int t32, hipStream_t st)
{
    if (n1 > n0)
        k_chunk_list<<<grid_for(n1 - n0, kListBlock), kListBlock, 0, st>>>(n0, n1, w.row, w.he, mark, epoch, lists,
                                                                           cap, cnt, t16, t32);
    k_chunk_info<<<1, 64, 0, st>>>(cnt, cap, info);
    return hipGetLastError();
}

hipError_t launch_sink_bands(const Inputs &in, const Work &w, int64_t n0, int64_t n1, int k_max, int32_t *strut_list,
                             int32_t *strut_cnt, const SinkOut &so, hipStream_t st)
{
    if (n1 > n0) {
        k_chunk_struts<<<grid_for(n1 - n0, kListBlock), kListBlock, 0, st>>>(n0, n1, w.row, w.he, w.node_rec,
                                                                             strut_list, strut_cnt);
        // a fixed grid of waves (enough to fill the chip) walks the strut
        // list; no more groups than the lattice has struts
        auto grid = [&](int g) {
            const int64_t groups = (in.n_struts + g - 1) / g;
            return (unsigned)(groups < kZipGrid ? (groups > 0 ? groups : 1) : kZipGrid);
        };
        // a band has about 2 (k + 4) samples
        if (k_max <= 24)
            k_sink_zip<8><<<grid(8), 64, 0, st>>>(w, so, strut_list, strut_cnt, in.sa, in.sb);
        else if (k_max <= 32)
            k_sink_zip<6><<<grid(6), 64, 0, st>>>(w, so, strut_list, strut_cnt, in.sa, in.sb);
        else if (k_max <= 56)
            k_sink_zip<4><<<grid(4), 64, 0, st>>>(w, so, strut_list, strut_cnt, in.sa, in.sb);
        else
            k_sink_zip<2><<<grid(2), 64, 0, st>>>(w, so, strut_list, strut_cnt, in.sa, in.sb);
    }
    return hipGetLastError();
}

hipError_t launch_sink_reduce(unsigned long long *slots, uint64_t *out, hipStream_t st)
{
    k_sink_reduce<<<1, 64, 0, st>>>(slots, out);
    return hipGetLastError();
}

hipError_t launch_range_done(int32_t *flags, int32_t *fail, int64_t r, hipStream_t st)
{
    k_range_done<<<1, 64, 0, st>>>(flags, fail, r);
    return hipGetLastError();
}

hipError_t launch_clear_parts(unsigned long long *slots, int64_t p0, int64_t p1, hipStream_t st)
{
    if (p1 > p0) k_clear_parts<<<grid_for((p1 - p0) * kSlots * kWords, 256), 256, 0, st>>>(slots, p0, p1);
    return hipGetLastError();
}

}  // namespace lm
