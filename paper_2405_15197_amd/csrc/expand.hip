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

__global__ void __launch_bounds__(64) k_expand(XParams P)
{
    __shared__ uint4 s_arc[kAcap][kRecArcFields / 4];  // the node's arcs, staged once
    __shared__ uint4 s_vtx[kVcap];                     // its vertices (name, xyz)
    const Work &W = P.w;
    const FillOut &O = P.o;
    const int64_t N = P.in.n_nodes;
    const int64_t n = xcd_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    if (n >= N) return;
    if (W.flags[0] & (DF_CAPACITY | DF_BADLAT | DF_RECCAP)) return;
    // the record's sizes are the node's counts: no wait for its header
    const int64_t rb = W.node_rec[n];
    const int64_t Np1 = N + 1;
    const int64_t voff = W.node_off[NC_VERT * Np1 + n], aoff = W.node_off[NC_ARC * Np1 + n];
    const int64_t hoff = W.node_off[NC_HOLE * Np1 + n];
    const int64_t moff = W.node_off[NC_MESH * Np1 + n], foff = W.node_off[NC_FAN * Np1 + n];
    const int V = (int)(W.node_off[NC_VERT * Np1 + n + 1] - voff);
    const int E = (int)(W.node_off[NC_ARC * Np1 + n + 1] - aoff);
    const int NC = (int)(W.node_off[NC_HOLE * Np1 + n + 1] - hoff);
    const int M = (int)(W.node_off[NC_MESH * Np1 + n + 1] - moff);
    const int F = (int)(W.node_off[NC_FAN * Np1 + n + 1] - foff);
    const float4 c4 = W.node4[n];
    if (rb < 0) return;
    const int wsum = M - NC;  // hole centres come last
    const uint32_t *R = W.rec + rb;
    const uint32_t *RV = R + kRecHead;
    const uint32_t *RA = RV + 4 * V;
    const uint32_t *RH = RA + kRecArcFields * E;
    // the node's Eq. 12 points follow its hole centres, by mesh index
    const uint32_t *RI = RH + 3 * NC - 3 * V;

    // arcs: whole 16-byte groups into LDS (the arc block starts on a 16-byte
    // boundary); every later read of an arc field is an LDS read.  The arcs
    // of a node of the multi-wave class (more than kAcap) stay in the record.
    const bool staged = E <= kAcap;
    if (staged)
        for (int x = lane; x < (kRecArcFields / 4) * E; x += 64)
            s_arc[x / (kRecArcFields / 4)][x % (kRecArcFields / 4)] = ((const uint4 *)RA)[x];
    const bool vstaged = V <= kVcap;
    if (vstaged)
        for (int i = lane; i < V; i += 64) s_vtx[i] = ((const uint4 *)RV)[i];
    __syncthreads();
    auto aw = [&](int j, int f) -> uint32_t {
        return staged ? ((const uint32_t *)s_arc[j])[f] : RA[kRecArcFields * j + f];
    };
    // word f (0 name, 1..3 xyz) of vertex i
    auto vw = [&](int i, int f) -> uint32_t {
        return vstaged ? ((const uint32_t *)&s_vtx[i])[f] : RV[4 * i + f];
    };
    if (O.vert_name) {
        for (int i = lane; i < V; i += 64) {
            O.vert_name[voff + i] = vw(i, 0);
            O.vert_xyz[0 * O.cap_vert + voff + i] = fbits(vw(i, 1));
            O.vert_xyz[1 * O.cap_vert + voff + i] = fbits(vw(i, 2));
            O.vert_xyz[2 * O.cap_vert + voff + i] = fbits(vw(i, 3));
        }
    }
    if (O.arc_f32) {
        const int64_t cA = O.cap_arc;
        for (int j = lane; j < E; j += 64) {
#pragma unroll
            for (int t = 0; t < 10; ++t) O.arc_f32[t * cA + aoff + j] = fbits(aw(j, t));
            O.arc_f32[10 * cA + aoff + j] = fbits(aw(j, 9)) + fbits(aw(j, 10));  // t2 = t1 + dt
            O.arc_u32[0 * cA + aoff + j] = aw(j, 11) & 0x1ffffu;  // p | q<<8 | whole<<16
            O.arc_u32[1 * cA + aoff + j] = aw(j, 12);
            O.arc_u32[2 * cA + aoff + j] = (uint32_t)n;
        }
    }
    __syncthreads();

    // mesh vertices: meta-vertices, interior points, hole centres
    for (int i = lane; i < M; i += 64) {
        float3 w;
        if (i < V) {
            w = make_float3(fbits(vw(i, 1)), fbits(vw(i, 2)), fbits(vw(i, 3)));
        } else if (i < wsum) {
            w = make_float3(fbits(RI[3 * i]), fbits(RI[3 * i + 1]), fbits(RI[3 * i + 2]));
        } else {
            const int c = i - wsum;
            w = make_float3(fbits(RH[3 * c]), fbits(RH[3 * c + 1]), fbits(RH[3 * c + 2]));
        }
        float *dst = O.mesh_xyz + 3 * (moff + i);
        dst[0] = c4.x + w.x;
        dst[1] = c4.y + w.y;
        dst[2] = c4.z + w.z;
    }
    // hole fans: one triangle per circular-arc segment, apex at the contour's
    // hole centre, oriented outward
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
    k_expand<<<(unsigned)in.n_nodes, 64, 0, st>>>(P);
    return hipGetLastError();
}

}  // namespace lm
