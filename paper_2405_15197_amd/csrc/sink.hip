// Sink mode: the lattice is meshed in chunks of node ids and the triangles
// are reduced to per-chunk counts and order-independent hashes instead of
// being stored (for lattices whose mesh does not fit in memory).
//
// A chunk is a node-id range [n0, n1).  Its node list is the range plus the
// halo: every neighbour with a higher id outside the range (the band of a
// strut is emitted by the chunk of its lower end, which needs the other
// end's loop).  Mesh vertices are named (node, node-local index), so the
// hashes do not depend on the chunking or on any global numbering:
//   vertex id   vid = node << 21 | local;
//   triangle    key = mix(mix(mix(v0 + G) ^ v1) ^ v2) with (v0, v1, v2) the
//               triangle's vids rotated so that the smallest comes first
//               (orientation kept), mix the SplitMix64 finaliser, G its
//               increment 0x9E3779B97F4A7C15;
//   vertex      key = mix(mix(mix(vid) ^ (bits(x) | bits(y) << 32)) ^ bits(z))
//               over the FP32 absolute position.
// Per chunk (LM_SINK_WORDS 64-bit words): triangles, sum of triangle keys,
// mesh vertices, sum of vertex keys, sums of round(x 2^20), round(y 2^20),
// round(z 2^20) (two's complement), nodes of the range without a mesh.
#include "common.h"

namespace lm {
namespace {

constexpr int kSlots = 64;  // spread of the hash atomics
constexpr int kWords = 8;

__device__ inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline uint64_t vid_of(int64_t node, int local) { return ((uint64_t)node << 21) | (uint64_t)local; }

__device__ inline uint64_t tri_key(uint64_t a, uint64_t b, uint64_t c)
{
    // rotate the smallest id first, keeping the cyclic order
    if (b < a && b < c) {
        const uint64_t t = a; a = b; b = c; c = t;
    } else if (c < a && c < b) {
        const uint64_t t = c; c = b; b = a; a = t;
    }
    return mix64(mix64(mix64(a + 0x9E3779B97F4A7C15ull) ^ b) ^ c);
}

__device__ inline uint64_t vert_key(uint64_t vid, float x, float y, float z)
{
    const uint64_t xy = (uint64_t)__float_as_uint(x) | ((uint64_t)__float_as_uint(y) << 32);
    return mix64(mix64(mix64(vid) ^ xy) ^ (uint64_t)__float_as_uint(z));
}

__device__ inline uint64_t wave_sum_u64(uint64_t x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

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

// Chunk node list in valence classes: the range, then the halo (marked
// with the chunk's epoch so that each halo node is listed once).
__global__ void __launch_bounds__(256) k_chunk_list(int64_t n0, int64_t n1, const int64_t *row, const int2 *he,
                                                    int32_t *mark, int32_t epoch, int32_t *lists, int64_t cap,
                                                    int32_t *cnt, int t16, int t32)
{
    const int64_t n = n0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = n < n1;
    int64_t r0 = 0, r1 = 0;
    if (in) {
        r0 = row[n];
        r1 = row[n + 1];
    }
    append(in, valence_class(r1 - r0, t16, t32), (int32_t)n, lists, cap, cnt);
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

struct SinkParams {
    Work w;
    int64_t N, n0, n1;
    unsigned long long *slots;  // [kSlots][kWords]
    const int32_t *node_part;   // per-part outputs when set
    unsigned long long *out_parts;
    const int64_t *part_base;   // first node of each part: vertex ids are part-local
};

__device__ inline int64_t local_node(const SinkParams &P, int64_t n)
{
    return P.node_part ? n - P.part_base[P.node_part[n]] : n;
}

// adds v to word `word` of the output of `part` (chunk mode: part is
// ignored); spread over kSlots slots by block to keep atomics apart
__device__ inline void add_out(const SinkParams &P, int32_t part, int word, uint64_t v)
{
    const int64_t slot = blockIdx.x & (kSlots - 1);
    if (P.node_part) atomicAdd(&P.out_parts[((int64_t)part * kSlots + slot) * kWords + word], (unsigned long long)v);
    else atomicAdd(&P.slots[slot * kWords + word], (unsigned long long)v);
}

// Mesh vertices and hole fans of the range's nodes, from their records.
__global__ void __launch_bounds__(64) k_sink_nodes(SinkParams P)
{
    __shared__ uint4 s_arc[kAcap][kRecArcFields / 4];  // the node's arcs, staged once
    const Work &W = P.w;
    const int64_t n = P.n0 + blockIdx.x;
    const int lane = threadIdx.x;
    if (n >= P.n1) return;
    const int64_t rb = W.node_rec[n];
    const int32_t part = P.node_part ? P.node_part[n] : 0;
    if (rb < 0) {
        if (lane == 0) add_out(P, part, 7, 1);
        return;
    }
    const uint32_t *R = W.rec + rb;
    const int V = (int)R[0], E = (int)R[1], NC = (int)R[2], ncirc = (int)R[3];
    const int wsum = (int)R[4], M = (int)R[5], F = (int)R[6];
    const uint32_t *RV = R + kRecHead;
    const uint32_t *RA = RV + 4 * V;
    const uint32_t *RH = RA + kRecArcFields * E;
    const float4 c4 = W.node4[n];
    const int64_t ln = local_node(P, n);
    // arcs: whole 16-byte groups into LDS; every arc field is then read there
    // (the arcs of a node of the multi-wave class stay in the record)
    const bool staged = E <= kAcap;
    if (staged)
        for (int x = lane; x < (kRecArcFields / 4) * E; x += 64)
            s_arc[x / (kRecArcFields / 4)][x % (kRecArcFields / 4)] = ((const uint4 *)RA)[x];
    __syncthreads();
    auto aw = [&](int j, int f) -> uint32_t {
        return staged ? ((const uint32_t *)s_arc[j])[f] : RA[kRecArcFields * j + f];
    };
    auto af = [&](int f, int j) { return __uint_as_float(aw(j, f)); };
    uint64_t hv = 0, sx = 0, sy = 0, sz = 0, ht = 0;
    for (int i = lane; i < M; i += 64) {
        float w0, w1, w2;
        if (i < V) {
            w0 = __uint_as_float(RV[4 * i + 1]);
            w1 = __uint_as_float(RV[4 * i + 2]);
            w2 = __uint_as_float(RV[4 * i + 3]);
        } else if (i < wsum) {
            int lo = 0, hi = E - 1;  // last arc with mbase <= i
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((int)aw(mid, 14) <= i) lo = mid;
                else hi = mid - 1;
            }
            const int nseg = (int)(aw(lo, 13) & 0xffffu);
            const bool fwd = (aw(lo, 11) >> 17) & 1u;
            const int jc = i - (int)aw(lo, 14);
            const int ii = fwd ? jc + 1 : nseg - 1 - jc;
            const float t1 = af(9, lo), t2 = af(10, lo);
            const float t = t1 + (t2 - t1) * (float)ii / (float)nseg;
            float s, c;
            sincosf(t, &s, &c);
            w0 = af(0, lo) + af(3, lo) * s + af(6, lo) * c;
            w1 = af(1, lo) + af(4, lo) * s + af(7, lo) * c;
            w2 = af(2, lo) + af(5, lo) * s + af(8, lo) * c;
        } else {
            const int c = i - wsum;
            w0 = __uint_as_float(RH[3 * c]);
            w1 = __uint_as_float(RH[3 * c + 1]);
            w2 = __uint_as_float(RH[3 * c + 2]);
        }
        const float x = c4.x + w0, y = c4.y + w1, z = c4.z + w2;
        hv += vert_key(vid_of(ln, i), x, y, z);
        sx += (uint64_t)llrint((double)x * 1048576.0);
        sy += (uint64_t)llrint((double)y * 1048576.0);
        sz += (uint64_t)llrint((double)z * 1048576.0);
    }
    for (int i = lane; i < F; i += 64) {
        int lo = 0, hi = ncirc - 1;  // last circular arc with fbase <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((int)aw(mid, 15) <= i) lo = mid;
            else hi = mid - 1;
        }
        const int j = lo;
        const uint32_t u0 = aw(j, 11), u1 = aw(j, 12), u2 = aw(j, 13);
        const bool fwd = (u0 >> 17) & 1u, lower = (u0 >> 18) & 1u;
        const int nseg = (int)(u2 & 0xffffu), contour = (int)(u2 >> 16);
        const int vs = (int)(u1 & 0xffffu), ve = (int)(u1 >> 16);
        const int mbase = (int)aw(j, 14);
        const int s = i - (int)aw(j, 15);
        const int i0 = fwd ? s : nseg - s, i1 = fwd ? s + 1 : nseg - s - 1;
        const int lo_i = i0 < i1 ? i0 : i1, hi_i = i0 < i1 ? i1 : i0;
        const int u = lo_i == 0 ? vs : mbase + (fwd ? lo_i - 1 : nseg - 1 - lo_i);
        const int u2i = hi_i == nseg ? ve : mbase + (fwd ? hi_i - 1 : nseg - 1 - hi_i);
        ht += tri_key(vid_of(ln, wsum + contour), vid_of(ln, lower ? u2i : u), vid_of(ln, lower ? u : u2i));
    }
    hv = wave_sum_u64(hv);
    sx = wave_sum_u64(sx);
    sy = wave_sum_u64(sy);
    sz = wave_sum_u64(sz);
    ht = wave_sum_u64(ht);
    if (lane == 0) {
        add_out(P, part, 0, (uint64_t)F);
        add_out(P, part, 1, ht);
        add_out(P, part, 2, (uint64_t)M);
        add_out(P, part, 3, hv);
        add_out(P, part, 4, sx);
        add_out(P, part, 5, sy);
        add_out(P, part, 6, sz);
    }
}

// Struts whose lower end is in the range and whose ends both have a mesh.
__global__ void __launch_bounds__(256) k_chunk_struts(int64_t n0, int64_t n1, const int64_t *row, const int2 *he,
                                                      const int64_t *node_rec, int32_t *list, int32_t *cnt)
{
    const int64_t n = n0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = n < n1;
    int64_t r0 = 0, r1 = 0;
    bool ok = false;
    if (in) {
        r0 = row[n];
        r1 = row[n + 1];
        ok = node_rec[n] >= 0;
    }
    int deg = (int)(r1 - r0);
    int maxdeg = deg;
    for (int o = 32; o > 0; o >>= 1) maxdeg = max(maxdeg, __shfl_xor(maxdeg, o, 64));
    for (int i = 0; i < maxdeg; ++i) {
        bool add = false;
        int32_t s = 0;
        if (i < deg && ok) {
            const int2 h = he[r0 + i];
            add = (int64_t)h.x > n && node_rec[h.x] >= 0;
            s = h.y;
        }
        append(add, 0, s, list, 0, cnt);
    }
}

// Bands of the listed struts (one wave per G), hashed.  A 4 KB staging
// buffer lets eight waves share a SIMD; G shrinks with the resolution so
// that a group's loops still fit it.
constexpr int kZipStage = 512;

template <int G>
__global__ void __launch_bounds__(64) k_sink_zip(SinkParams P, const int32_t *list, const int32_t *cnt,
                                                 const int32_t *sa, const int32_t *sb)
{
    __shared__ int2 st[kZipStage];
    __shared__ int g_na[G], g_nb[G], g_ra[G], g_rb[G];
    __shared__ int64_t g_la[G], g_lb[G], g_a[G], g_b[G];
    __shared__ int g_t[G + 1];
    __shared__ unsigned long long g_h[G];  // triangle-key sum per strut
    const Work &W = P.w;
    const int lane = threadIdx.x;
    const int64_t ns_all = *cnt;
    const int64_t g0 = (int64_t)blockIdx.x * G;
    if (g0 >= ns_all) return;
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
        // sorted-order views of both loops (LDS when staged)
        auto A = [&](int k) -> int2 {
            if (staged) return st[g_t[i] + k];
            int q = ra + k;
            return loops[g_la[i] + (q >= na ? q - na : q)];
        };
        auto B = [&](int k) -> int2 {
            if (staged) return st[g_t[i] + na + k];
            int q = rb + k;
            return loops[g_lb[i] + (q >= nb ? q - nb : q)];
        };
        auto pred = [&](bool onB, float xv, bool inclusive) {
            const int n = onB ? nb : na;
            int lo = 0, hi = n;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const float p = __int_as_float((onB ? B(mid) : A(mid)).y);
                if (inclusive ? (p <= xv) : (p < xv)) lo = mid + 1;
                else hi = mid;
            }
            return lo == 0 ? n - 1 : lo - 1;
        };
        const int64_t na_node = local_node(P, g_a[i]), nb_node = local_node(P, g_b[i]);
        if (j < na) {
            int k0 = j - ra;
            if (k0 < 0) k0 += na;
            const int k1 = k0 + 1 == na ? 0 : k0 + 1;
            const int2 u = A(k0), u2 = A(k1);
            const int ap = pred(true, __int_as_float(u2.y), false);
            ht += tri_key(vid_of(na_node, u.x), vid_of(na_node, u2.x), vid_of(nb_node, B(ap).x));
        } else {
            int k0 = j - na - rb;
            if (k0 < 0) k0 += nb;
            const int k1 = k0 + 1 == nb ? 0 : k0 + 1;
            const int2 w = B(k0), w2 = B(k1);
            const int ap = pred(false, __int_as_float(w2.y), true);
            ht += tri_key(vid_of(nb_node, w2.x), vid_of(nb_node, w.x), vid_of(na_node, A(ap).x));
        }
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
                add_out(P, cur, 0, cnt_s);
                add_out(P, cur, 1, h_s);
                cur = pt;
                cnt_s = h_s = 0;
            }
            cnt_s += (uint64_t)(g_t[i + 1] - g_t[i]);
            h_s += g_h[i];
        }
        add_out(P, cur, 0, cnt_s);
        add_out(P, cur, 1, h_s);
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
        k_chunk_list<<<grid_for(n1 - n0, 256), 256, 0, st>>>(n0, n1, w.row, w.he, mark, epoch, lists, cap, cnt, t16,
                                                             t32);
    k_chunk_info<<<1, 64, 0, st>>>(cnt, cap, info);
    return hipGetLastError();
}

hipError_t launch_sink(const Inputs &in, const Work &w, int64_t n0, int64_t n1, int64_t max_struts, int k_max,
                       int32_t *strut_list, int32_t *strut_cnt, unsigned long long *slots, uint64_t *out,
                       const int32_t *node_part, uint64_t *out_parts, const int64_t *part_base, hipStream_t st)
{
    SinkParams P;
    P.w = w;
    P.N = in.n_nodes;
    P.n0 = n0;
    P.n1 = n1;
    P.slots = slots;
    P.node_part = node_part;
    P.out_parts = (unsigned long long *)out_parts;
    P.part_base = part_base;
    if (n1 > n0) {
        k_sink_nodes<<<(unsigned)(n1 - n0), 64, 0, st>>>(P);
        k_chunk_struts<<<grid_for(n1 - n0, 256), 256, 0, st>>>(n0, n1, w.row, w.he, w.node_rec, strut_list,
                                                                 strut_cnt);
        // grid for the most struts the range can own (its half-edges)
        if (max_struts > 0) {
            // a band has about 2 (k + 4) samples
            if (k_max <= 24)
                k_sink_zip<8><<<grid_for(max_struts, 8), 64, 0, st>>>(P, strut_list, strut_cnt, in.sa, in.sb);
            else if (k_max <= 56)
                k_sink_zip<4><<<grid_for(max_struts, 4), 64, 0, st>>>(P, strut_list, strut_cnt, in.sa, in.sb);
            else
                k_sink_zip<2><<<grid_for(max_struts, 2), 64, 0, st>>>(P, strut_list, strut_cnt, in.sa, in.sb);
        }
    }
    if (!node_part) k_sink_reduce<<<1, 64, 0, st>>>(slots, out);
    return hipGetLastError();
}

}  // namespace lm
