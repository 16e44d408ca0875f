// Internal declarations shared by the latmesh HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lm {

// Per-node limits of this library.  Nodes of up to kVmax incident struts are
// meshed by one wave (or a part of one); nodes of kVmax + 1 .. kVmaxBig by a
// group of kBigWaves waves sharing the node's LDS.  A node beyond the limits
// is flagged (its status bit is set) and emits nothing.
// FP32 -> FP64 hand-over beside the condition number (kappa_max): a seam
// conic whose centre or semi-major axis exceeds kConicMax rho, or a vertex
// whose FP32 error bound exceeds kVertexErr rho (kFp32Eps: unit roundoff).
constexpr float kConicMax = 4.0f;
constexpr float kVertexErr = 4e-6f;
constexpr float kFp32Eps = 5.9604645e-8f;
constexpr int kVmax = 16;       // incident struts per node, one-wave classes
constexpr int kAcap = 64;       // arcs per node, one-wave classes
constexpr int kVcap = 64;       // meta-vertices per node, one-wave classes
constexpr int kVmaxBig = 64;    // incident struts per node, multi-wave class
constexpr int kAcapBig = 192;   // arcs per node, multi-wave class
constexpr int kVcapBig = 128;   // meta-vertices per node, multi-wave class
constexpr int kBigWaves = 4;    // waves per node of the multi-wave class
// The FP64 pass splits the multi-wave class: nodes of kVmax + 1 .. kVmaxMid
// struts run on two waves with capacities for that many (a node that does
// not fit them goes on to the four-wave kernel), larger ones on four.
constexpr int kVmaxMid = 32;
constexpr int kAcapMid = 96;
constexpr int kVcapMid = 64;
constexpr int kPieces = 4;      // kept arcs per conic

constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInvTwoPi = 0.159154943091895335769f;

enum NodeStatus : int {
    NS_INVALID_STRUT = 1,
    NS_NON_ELLIPTIC = 2,
    NS_LOOP = 4,
    NS_TOPOLOGY = 8,
    NS_ISOLATED = 16,
    NS_VALENCE = 32,
    NS_DUPLICATE = 64,
    NS_CAPACITY = 128,
    NS_PREC = 256,  // internal: FP32 result not trusted, redo in FP64
};

// Per-node count columns (int32, field-major [kNodeCols][N]).
enum NodeCol : int {
    NC_VERT = 0,
    NC_ARC = 1,
    NC_HOLE = 2,
    NC_MESH = 3,
    NC_FAN = 4,
    NC_STATUS = 5,
    kNodeCols = 6,
};
constexpr int kNodeScanCols = 5;  // columns 0..4 are prefix-summed

// Device-side flag words: flags[0] DevFlag bits of the last count / fill,
// flags[1] DevFlag bits of the lattice preparation, flags[2] number of nodes
// handed to the FP64 pass.
enum DevFlag : int {
    DF_CAPACITY = 1,   // an output was too small, writes skipped
    DF_BADLAT = 4,     // a strut endpoint is out of range
    DF_RECCAP = 8,     // node-record space too small, or mesh too large for int32
};

// Node records.  The count pass leaves every meshed node's result in the
// record space, 32-bit words, allocated in kRecRegions regions (node n uses
// region n mod kRecRegions, each with its own bump counter):
//   header  [kRecHead]  V, E, H (holes), ncirc (circular arcs, stored first),
//                       wsum (first hole-centre mesh index), M (mesh
//                       vertices), F (fan triangles), 0
//   vertices [V][4]     name, x, y, z (node-local), one 16-byte group each
//   arcs    [E][16]     o.xyz, a.xyz, b.xyz, t1, dt = t2 - t1 (float bits),
//                       p | q<<8 | whole<<16 | fwd<<17 | lower<<18,
//                       vs | ve<<16, nseg | contour<<16, mbase, fbase: four
//                       16-byte groups each
//   holes   [H][3]      hole centres (node-local)
//   points  [wsum-V][3] the Eq. 12 interior points (node-local, in mesh
//                       order), as the node's precision computed them; the
//                       loop table starts at rec_table_word(V, E, H + wsum - V)
//                       (not in sink mode, whose records hold the loops only)
//   loop table          bytes: loop start of each strut label 1..v+1 (v+1
//                       bytes), then for every loop entry in loop order its
//                       arc | 0x80 if the arc runs along the loop (header
//                       word 7 = v | entries << 8 | fp64 << 24 | wide << 25,
//                       fp64 set when the node was meshed in FP64; wide: the
//                       node has more than 127 arcs or 255 loop entries
//                       possible (multi-wave class), and the table holds
//                       16-bit entries, the direction in bit 15)
//   loops               from a multiple of 4 words: for each incident strut
//                       in label order, its end loop as int2 (node-local mesh
//                       vertex, phi bits), in loop order
// fwd: the arc is subdivided from t1 (its smaller-name end is at t1);
// lower: the arc's strut q runs to a higher node id.
constexpr int kRecHead = 8;
constexpr int kRecArcFields = 16;
constexpr int kRecRegions = 128;
__host__ __device__ inline int64_t rec_table_word(int V, int E, int H)
{
    return (int64_t)kRecHead + 4 * V + kRecArcFields * E + 3 * H;
}
__host__ __device__ inline int64_t rec_loop_word(int V, int E, int H, int table_bytes)
{
    return (rec_table_word(V, E, H) + (table_bytes + 3) / 4 + 3) & ~(int64_t)3;
}
// bytes of the loop table of a node of valence v with nent loop entries
__host__ __device__ inline int rec_table_bytes(int v, int nent, bool wide)
{
    return (wide ? 2 : 1) * (v + 1 + nent);
}
constexpr uint32_t kRecFp64 = 1u << 24;  // header word 7: meshed in FP64
constexpr uint32_t kRecWide = 1u << 25;  // header word 7: 16-bit loop table

struct Inputs {
    int64_t n_nodes, n_struts;
    const float *x, *y, *z, *r;
    const int32_t *sa, *sb;
};

// Workspace pointers (device).
struct Work {
    float4 *node4;          // [N] x, y, z, radius
    int64_t *row;           // [N+1] adjacency offsets
    int2 *he;               // [2S] (far node, strut id), strut id ascending per node
    int32_t *deg;           // [N] scratch: degree / fill cursor
    int64_t *strut_he;      // [2S] half-edge index at the lower / higher node id
    int32_t *node_cnt;      // [kNodeCols][N]
    int64_t *node_off;      // [kNodeScanCols][N+1]
    int32_t *he_len;        // [2S] loop samples per half-edge
    int64_t *he_loop;       // [2S] first loop sample (int2 index into rec)
    int32_t *he_rot;        // [2S] loop position of the smallest phi
    int32_t *band_cnt;      // [S]
    int64_t *band_off;      // [S+1]
    int64_t *node_rec;      // [N] first word of the node's record, -1: none
    uint32_t *rec;          // node records (see above)
    int64_t rec_words;      // capacity in words (kRecRegions equal regions)
    unsigned long long *rec_top;  // [kRecRegions] words used per region
    int64_t *scan_tmp;      // block partials
    int64_t scan_tmp_len;
    int32_t *flags;         // [4] see DevFlag
    int64_t *totals;        // [16] device copy of totals
    int32_t *fb_list;       // [N] nodes for the FP64 pass
    int32_t *queue;         // [N] node ids grouped by valence class
    int64_t *cls_info;      // [8] nodes per class (0..3), queue start per class (4..7)
    int32_t *work_ctr;      // [8] work counters: FP32 classes 0..3, FP64 passes 4 (one wave), 5 (four waves) and 6 (two waves)
    const int16_t *node_k;  // [N] per-node resolution (batched parts) or null
    // adjoint scratch (set before lm_loss / lm_backward run)
    double *loss_node;      // [N][3] loss terms per node
    float *grad_node;       // [N][4] adjoint of each node's own x, y, z, radius
    float *grad_he;         // [2S][4] adjoint of the far node's inputs, per half-edge
};

// Workgroups are dispatched to the 8 XCDs (each with its own L2) in turn:
// block b runs on XCD b % 8.  This maps the blocks of one XCD to one
// contiguous range of [0, nb), so that each L2 sees whole output lines.
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t x = b % kXcds, q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// Valence classes of the node kernel: v <= 4 (four nodes per wave), 5..8
// (two per wave), 9..kVmax (one per wave), otherwise (kBigWaves waves per
// node).  The batched entry point may lower the first two limits (4 and 8
// are the class capacities).
__host__ __device__ inline int valence_class(int64_t v, int t16 = 4, int t32 = 8)
{
    return v <= t16 ? 0 : (v <= t32 ? 1 : (v <= kVmax ? 2 : 3));
}
constexpr int kClasses = 4;

// sin and cos of x in FP32 for every FP32 pass (one definition, so the node
// pass, the expansion, sink-mode hashing and the adjoint evaluate the same
// points).  Cody and Waite's reduction by pi/2 (x = q pi/2 + r, |r| <= pi/4,
// pi/2 split into two FP32 constants applied with fused multiply-adds),
// then the Taylor series of sin to degree 9 and of cos to degree 10 on r
// (truncation below 3e-9) and the quadrant's sign and swap.  Absolute error
// within about one FP32 ulp of 1 for |x| < 2^13 (measured against FP64
// sin / cos, like the library's); the reduction loses about q * 4e-15 more
// beyond that.  The callers' arguments are arc parameters of a few turns.
__device__ __forceinline__ void sincos_f32(float x, float *s, float *c)
{
    constexpr float kTwoOverPi = 0.636619772f;
    constexpr float kHalfPi1 = 1.57079637f;      // pi/2 rounded to FP32
    constexpr float kHalfPi2 = -4.37113883e-8f;  // pi/2 - kHalfPi1
    const float q = rintf(x * kTwoOverPi);
    float r = fmaf(-q, kHalfPi1, x);
    r = fmaf(-q, kHalfPi2, r);
    const float r2 = r * r;
    float ps = fmaf(r2, 2.75573192e-6f, -1.98412698e-4f);  // 1/9!, -1/7!
    ps = fmaf(r2, ps, 8.33333333e-3f);                      // 1/5!
    ps = fmaf(r2, ps, -1.66666667e-1f);                     // -1/3!
    const float sn = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, -2.75573192e-7f, 2.48015873e-5f);  // -1/10!, 1/8!
    pc = fmaf(r2, pc, -1.38888889e-3f);                     // -1/6!
    pc = fmaf(r2, pc, 4.16666667e-2f);                      // 1/4!
    pc = fmaf(r2, pc, -0.5f);                               // -1/2!
    const float cs = fmaf(r2, pc, 1.0f);
    const int i = (int)q & 3;
    const float a = (i & 1) ? cs : sn, b = (i & 1) ? sn : cs;
    *s = (i & 2) ? -a : a;
    *c = ((i + 1) & 2) ? -b : b;
}

// Eq. 12 point ii (of nseg segments) of an arc x(t) = o + a sin t + b cos t,
// t in [t1, t1 + dt], node-local, from FP32 fields.  A whole conic (no end
// points) is evaluated directly.  An arc is evaluated from its start point
// x1 = x(t1) (its vertex) as x1 + a (sin t - sin t1) + b (cos t - cos t1),
// the differences in product form, 2 cos(t1 + h) sin h and
// -2 sin(t1 + h) sin h with h = (t - t1) / 2: a point of a long, thin seam
// ellipse (|a| far above the node radius, the arc a short piece of it near
// the node) then carries rounding relative to its distance from x1 rather
// than to |a|.  The one formula of every pass that outputs mesh vertices
// (stored mode and sink mode give the same bits).
__device__ __forceinline__ float3 arc_point_f32(const float *o, const float *a, const float *b, const float *x1,
                                                float t1, float dt, int ii, int nseg, bool whole)
{
    if (whole) {
        const float t = t1 + dt * (float)ii / (float)nseg;
        float s, c;
        sincos_f32(t, &s, &c);
        return make_float3(o[0] + a[0] * s + b[0] * c, o[1] + a[1] * s + b[1] * c, o[2] + a[2] * s + b[2] * c);
    }
    const float h = 0.5f * dt * (float)ii / (float)nseg;
    float sh, ch, sm, cm;
    sincos_f32(h, &sh, &ch);
    sincos_f32(t1 + h, &sm, &cm);
    const float ds = 2.f * cm * sh, dc = -2.f * sm * sh;
    return make_float3(x1[0] + a[0] * ds + b[0] * dc, x1[1] + a[1] * ds + b[1] * dc, x1[2] + a[2] * ds + b[2] * dc);
}

// ---- sink mode: counts and order-independent hashes instead of a mesh ----
// A mesh vertex is named vid = node << 21 | node-local index; a triangle's
// key is mix(mix(mix(v0 + G) ^ v1) ^ v2) with its vids rotated so that the
// smallest comes first (orientation kept), a vertex's key
// mix(mix(mix(vid) ^ (bits(x) | bits(y) << 32)) ^ bits(z)) over its FP32
// absolute position; mix is the SplitMix64 finaliser, G its increment.
// Sums are modulo 2^64, so they do not depend on chunking or numbering.
constexpr int kSinkSlots = 64;  // spread of the hash atomics
constexpr int kSinkWords = 8;   // triangles, triangle keys, mesh vertices, vertex keys,
                                // fixed-point x, y, z sums, nodes without a mesh

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

// Where sink-mode words go: per chunk through slots (node_part null), or per
// part (the part of a node from node_part, vertex ids local to the part).
// The node pass counts vertices and fans of the nodes in [n0, n1) only (the
// chunk's own nodes; its halo is meshed for the bands' loops).
struct SinkOut {
    int64_t n0, n1;
    unsigned long long *slots;      // [kSinkSlots][kSinkWords]
    const int32_t *node_part;       // [N] or null
    unsigned long long *out_parts;  // [parts][kSinkSlots][kSinkWords]
    const int64_t *part_base;       // first node of each part
};

__device__ inline int64_t sink_local_node(const SinkOut &S, int64_t n)
{
    return S.node_part ? n - S.part_base[S.node_part[n]] : n;
}

// adds v to word `word` of `part`'s output (chunk mode: part ignored),
// spread over kSinkSlots slots by block
__device__ inline void sink_add(const SinkOut &S, int32_t part, int word, uint64_t v)
{
    const int64_t slot = blockIdx.x & (kSinkSlots - 1);
    if (S.node_part)
        atomicAdd(&S.out_parts[((int64_t)part * kSinkSlots + slot) * kSinkWords + word], (unsigned long long)v);
    else
        atomicAdd(&S.slots[slot * kSinkWords + word], (unsigned long long)v);
}

struct FillOut {
    float *mesh_xyz;
    int32_t *tri;
    int64_t cap_mesh, cap_tri;
    uint32_t *vert_name;
    float *vert_xyz;
    int64_t cap_vert;
    float *arc_f32;
    uint32_t *arc_u32;
    int64_t cap_arc;
};

// launchers (return hipError_t)
hipError_t launch_prepare(const Inputs &in, const Work &w, hipStream_t st);
// node radii from per-strut end radii [S][2] (mean per node, mismatches
// beyond rel_tol counted), and the end-radius gradient [S][2] of a node-radius
// gradient; both need the adjacency of launch_prepare
hipError_t launch_end_radii(const Inputs &in, const Work &w, const float *end_r, float rel_tol, float *radius,
                            int32_t *mismatch, hipStream_t st);
hipError_t launch_end_grad(const Inputs &in, const Work &w, const float *grad_r, float *grad_end, hipStream_t st);
hipError_t launch_scan(const int32_t *src, int64_t *dst, int64_t n, int ncols, int64_t src_stride,
                       int64_t dst_stride, int64_t *tmp, int64_t tmp_len, hipStream_t st);
// Per-node meta-meshing (counts and node records), FP32 over all nodes or
// FP64 over the hand-over list.
// With src_rec set, the meta-mesh of each node is read from its record in
// src_rec (src_node_rec) and only re-subdivided at resolution k.
// src_rec / src_node_rec set: re-subdivision of the meta-mesh in those
// records; nodes that must be solved in full go to redo ([N], partitioned
// like the queue) with counts and work counters in redo_cnt [8], zeroed by
// the caller.
// Thread-centric ablation of the FP32 node pass (one lane per node, node id
// order, per-node scratch of node_thread_scratch_bytes() in global memory).
size_t node_thread_scratch_bytes();
hipError_t launch_node_thread(const Inputs &in, const Work &w, int k, float kappa_max, void *scratch,
                              hipStream_t st);

// Arc codec (encode: arc + u32 -> codes, mask, fallback; decode: codes ->
// out), one thread per arc.
hipError_t launch_arc_codec(const Inputs &in, const Work &w, bool encode, const float *arc, const uint32_t *u32,
                            int64_t E, int64_t ld, double rmin, double rmax, uint32_t *codes, uint32_t *mask,
                            float *fb, int64_t fb_cap, unsigned long long *fb_n, float *out, int64_t ld_out,
                            hipStream_t st);
// With sink set, the node pass runs in sink mode (end loops only in the
// records; vertices and fans of the nodes in [sink->n0, sink->n1) hashed).
// cls_est (host, may be null): nodes per valence class as last read back,
// used only to size the persistent grids (any size covers every queued node).
hipError_t launch_node(const Inputs &in, const Work &w, int k, float kappa_max, int fp64, hipStream_t st,
                       const uint32_t *src_rec = nullptr, const int64_t *src_node_rec = nullptr,
                       int32_t *redo = nullptr, int32_t *redo_cnt = nullptr, const SinkOut *sink = nullptr,
                       const int64_t *cls_est = nullptr);
// Node records -> meta-mesh, mesh vertices and hole fans.
hipError_t launch_expand(const Inputs &in, const Work &w, const FillOut &o, hipStream_t st);
hipError_t launch_band_count(const Inputs &in, const Work &w, hipStream_t st);
// bands; k (the resolution) sizes the groups of struts per wave
hipError_t launch_zip(const Inputs &in, const Work &w, const FillOut &o, int k, hipStream_t st);
hipError_t launch_totals(const Inputs &in, const Work &w, const FillOut *o, hipStream_t st);
// Loss terms (area, volume about p0, sum of squared norms) of the last mesh
// and their gradient dldx [cap_mesh][3]; then the adjoint to the inputs.
hipError_t launch_loss(const Inputs &in, const Work &w, const FillOut &o, float3 p0, float w_area, float w_vol,
                       float w_sq, float *dldx, double *terms, hipStream_t st);
hipError_t launch_backward(const Inputs &in, const Work &w, const float *dldx, float *grad_xyz, float *grad_r,
                           hipStream_t st);
// Sink mode: chunk node lists (range + higher-id halo, in valence classes)
// and the hashed triangles of a range.
int64_t sink_slots_words();  // per chunk or per part
hipError_t launch_parts_reduce(const unsigned long long *slots, int64_t n_parts, uint64_t *out, hipStream_t st);
hipError_t launch_part_map(int64_t N, const int64_t *part_off, const int32_t *part_k, int64_t n_parts,
                           int32_t *node_part, int16_t *node_k, hipStream_t st);
hipError_t launch_chunk_list(const Work &w, int64_t n0, int64_t n1, int32_t *mark, int32_t epoch, int32_t *lists,
                             int64_t cap, int32_t *cnt, int64_t *info, int t16, int t32, hipStream_t st);
// The struts a range owns (lower end in [n0, n1), both ends meshed) and their
// bands, hashed into `so`'s slots; k_max: the largest resolution among the
// range's nodes (sizes the groups of struts per wave).
hipError_t launch_sink_bands(const Inputs &in, const Work &w, int64_t n0, int64_t n1, int k_max, int32_t *strut_list,
                             int32_t *strut_cnt, const SinkOut &so, hipStream_t st);
// chunk slots -> out[kSinkWords]; clears the slots
hipError_t launch_sink_reduce(unsigned long long *slots, uint64_t *out, hipStream_t st);
// after range r's node pass: fail[r] = records overflowed; flags cleared
hipError_t launch_range_done(int32_t *flags, int32_t *fail, int64_t r, hipStream_t st);
// zero the per-part slots of parts [p0, p1)
hipError_t launch_clear_parts(unsigned long long *slots, int64_t p0, int64_t p1, hipStream_t st);

int64_t scan_tmp_needed(int64_t n, int ncols);

}  // namespace lm
