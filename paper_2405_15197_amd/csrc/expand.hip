// Expansion of the node records into the outputs: meta-mesh vertices and
// arcs (Sec. 4.2 stores them per node), the triangle-mesh vertices — the
// meta-vertices, the Eq. 12 interior points of every arc and one Eq. 13 hole
// centre per hole contour — and the hole fans (Sec. 5).  One wave per node;
// every store of a wave goes to consecutive addresses.
#include "common.h"

namespace lm {
namespace {

struct XParams {
    Inputs in;
    Work w;
    FillOut o;
};

__device__ inline float fbits(uint32_t u) { return __uint_as_float(u); }

// Mesh vertex i of the node (node-local): a meta-vertex (record word 1..3 of
// its 16-byte group), an Eq. 12 point (by mesh index, after the hole
// centres) or a hole centre
__device__ inline float3 mesh_local(const uint32_t *RV, const uint32_t *RI, const uint32_t *RH, int V, int wsum,
                                    int i)
{
    const uint32_t *src = i < V ? RV + 4 * i + 1 : (i < wsum ? RI + 3 * i : RH + 3 * (i - wsum));
    return make_float3(fbits(src[0]), fbits(src[1]), fbits(src[2]));
}

// The latency of the node's loads bounds this kernel (a few KB per node): the
// bookkeeping words are loaded together, then the first item of each output
// per lane (one round for most nodes) before any store, so that one wait
// covers all of them.  Two nodes per block, one per wave (half the blocks to
// dispatch).
__global__ void __launch_bounds__(128) k_expand(XParams P)
{
    __shared__ uint4 s_arc[2][kAcap][2];  // per wave: words 8..15 of each arc, for the hole fans
    const Work &W = P.w;
    const FillOut &O = P.o;
    const int64_t N = P.in.n_nodes;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int64_t n = 2 * xcd_block(blockIdx.x, gridDim.x) + wv;
    const bool live = n < N;
    const int64_t nn = live ? n : 0;
    // the record's sizes are the node's counts: no wait for its header
    const int flags = W.flags[0];
    const int64_t rb = W.node_rec[nn];
    const int64_t Np1 = N + 1;
    const int64_t voff = W.node_off[NC_VERT * Np1 + nn], aoff = W.node_off[NC_ARC * Np1 + nn];
    const int64_t hoff = W.node_off[NC_HOLE * Np1 + nn];
    const int64_t moff = W.node_off[NC_MESH * Np1 + nn], foff = W.node_off[NC_FAN * Np1 + nn];
    const int V = (int)(W.node_off[NC_VERT * Np1 + nn + 1] - voff);
    const int E = (int)(W.node_off[NC_ARC * Np1 + nn + 1] - aoff);
    const int NC = (int)(W.node_off[NC_HOLE * Np1 + nn + 1] - hoff);
    const int M = (int)(W.node_off[NC_MESH * Np1 + nn + 1] - moff);
    const int F = (int)(W.node_off[NC_FAN * Np1 + nn + 1] - foff);
    const float4 c4 = W.node4[nn];
    const bool go = live && !(flags & (DF_CAPACITY | DF_BADLAT | DF_RECCAP)) && rb >= 0;
    const int wsum = M - NC;  // hole centres come last
    const uint32_t *R = W.rec + (go ? rb : 0);
    const uint32_t *RV = R + kRecHead;
    const uint32_t *RA = RV + 4 * V;
    const uint32_t *RH = RA + kRecArcFields * E;
    // the node's Eq. 12 points follow its hole centres, by mesh index
    const uint32_t *RI = RH + 3 * NC - 3 * V;
    const uint4 *RA4 = (const uint4 *)RA;  // the arc block starts on a 16-byte boundary
    const bool want_arcs = O.arc_f32 != nullptr || F > 0;
    const int64_t cA = O.cap_arc;

    auto put_mesh = [&](int i, float3 w) {
        float *dst = O.mesh_xyz + 3 * (moff + i);
        dst[0] = c4.x + w.x;
        dst[1] = c4.y + w.y;
        dst[2] = c4.z + w.z;
    };
    auto put_vert = [&](int i, uint4 g) {
        O.vert_name[voff + i] = g.x;
        O.vert_xyz[0 * O.cap_vert + voff + i] = fbits(g.y);
        O.vert_xyz[1 * O.cap_vert + voff + i] = fbits(g.z);
        O.vert_xyz[2 * O.cap_vert + voff + i] = fbits(g.w);
    };
    auto put_arc = [&](int j, uint4 g0, uint4 g1, uint4 g2, uint4 g3) {
        const uint32_t f[13] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w, g2.x, g2.y, g2.z, g2.w, g3.x};
#pragma unroll
        for (int t = 0; t < 10; ++t) O.arc_f32[t * cA + aoff + j] = fbits(f[t]);
        O.arc_f32[10 * cA + aoff + j] = fbits(f[9]) + fbits(f[10]);  // t2 = t1 + dt
        O.arc_u32[0 * cA + aoff + j] = f[11] & 0x1ffffu;              // p | q<<8 | whole<<16
        O.arc_u32[1 * cA + aoff + j] = f[12];
        O.arc_u32[2 * cA + aoff + j] = (uint32_t)n;
    };

    uint4 g2 = make_uint4(0, 0, 0, 0), g3 = g2;
    if (go) {
        // first round: item `lane` of every output, all loads before any store
        float3 w0 = make_float3(0.f, 0.f, 0.f);
        uint4 g0 = g2, g1 = g2, gv = g2;
        if (lane < M) w0 = mesh_local(RV, RI, RH, V, wsum, lane);
        if (want_arcs && lane < E) {
            g0 = RA4[4 * lane];
            g1 = RA4[4 * lane + 1];
            g2 = RA4[4 * lane + 2];
            g3 = RA4[4 * lane + 3];
        }
        if (O.vert_name && lane < V) gv = ((const uint4 *)RV)[lane];
        if (lane < M) put_mesh(lane, w0);
        if (O.arc_f32 && lane < E) put_arc(lane, g0, g1, g2, g3);
        if (O.vert_name && lane < V) put_vert(lane, gv);
        // further rounds (nodes with more than 64 of an item)
        for (int i = lane + 64; i < M; i += 64) put_mesh(i, mesh_local(RV, RI, RH, V, wsum, i));
        if (O.arc_f32)
            for (int j = lane + 64; j < E; j += 64) put_arc(j, RA4[4 * j], RA4[4 * j + 1], RA4[4 * j + 2], RA4[4 * j + 3]);
        if (O.vert_name)
            for (int i = lane + 64; i < V; i += 64) put_vert(i, ((const uint4 *)RV)[i]);
    }
    // hole fans: one triangle per circular-arc segment, apex at the contour's
    // hole centre, oriented outward.  Words 8..15 of the arcs go to the wave's
    // LDS (the arcs of a multi-wave-class node, more than kAcap, stay in the
    // record).  Both waves of the block reach the barrier.
    const bool fans = go && F > 0;
    const bool staged = E <= kAcap;
    if (fans && staged && lane < E) {
        s_arc[wv][lane][0] = g2;
        s_arc[wv][lane][1] = g3;
    }
    __syncthreads();
    if (!fans) return;
    auto aw = [&](int j, int f) -> uint32_t {  // word f (8..15) of arc j
        return staged ? ((const uint32_t *)s_arc[wv][j])[f - 8] : RA[kRecArcFields * j + f];
    };
    const int64_t fan0 = W.band_off[P.in.n_struts] + foff;
    for (int i = lane; i < F; i += 64) {
        // last arc with fbase <= i: a circular arc (the others, after them,
        // have fbase = F)
        int lo = 0, hi = E - 1;
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
        // interior point ii sits at mbase + (fwd ? ii - 1 : nseg - 1 - ii)
        const int u = lo_i == 0 ? vs : mbase + (fwd ? lo_i - 1 : nseg - 1 - lo_i);
        const int u2i = hi_i == nseg ? ve : mbase + (fwd ? hi_i - 1 : nseg - 1 - hi_i);
        int32_t *t = O.tri + 3 * (fan0 + i);
        t[0] = (int32_t)(moff + wsum + contour);
        t[1] = (int32_t)(moff + (lower ? u2i : u));
        t[2] = (int32_t)(moff + (lower ? u : u2i));
    }
}

}  // namespace

hipError_t launch_expand(const Inputs &in, const Work &w, const FillOut &o, hipStream_t st)
{
    if (in.n_nodes == 0) return hipSuccess;
    XParams P;
    P.in = in;
    P.w = w;
    P.o = o;
    k_expand<<<(unsigned)((in.n_nodes + 1) / 2), 128, 0, st>>>(P);
    return hipGetLastError();
}

}  // namespace lm
