// Per-node meta-meshing and node-local triangulation (one wave per node).
//
// Geometry (Sec. 4.1, Sec. 4.3.1): around node c with nodal-sphere radius rho,
// incident strut m (far node c_m, radius rho_m, L = |c_m - c|) has
//   e_m = (c_m - c)/L, sigma_m = (rho - rho_m)/L, kappa_m = sqrt(1 - sigma_m^2)
// and the affine function P_m(w) = g_m . w - h_m (w = x - c) with
// g_m = e_m / kappa_m, h_m = rho sigma_m / kappa_m: the arc length along a
// generator of the tangent cone, measured from the tangency circle.  Cone m
// is |w|^2 - rho^2 = P_m^2, two cones meet on the auxiliary plane P_p = P_q,
// and the surface near the node is |w|^2 - rho^2 = max(0, P_1..P_v)^2.
// Label 0 stands for the nodal sphere (P_0 = 0).
//
// Work per node, lanes over the v(v+1)/2 conics (p, q), p < q, in
// lexicographic order:
//   1. conic: the tangency circle for (0, q); for p >= 1 the section of cone
//      p by its auxiliary plane with q, in principal axes (the ellipse of
//      Eq. 7, obtained here by completing the square in the plane);
//   2. trimming (Eqs. 8-9): keep P_p >= P_r for every other label r; each r
//      gives R cos(t - psi) >= -C, one circular interval; the intervals are
//      intersected in registers into at most kPieces arcs;
//   3. arc ends are triple ties (p, q, r); the tie point's rank along
//      (g_p - g_q) x (g_p - g_r) comes from the chord direction of the
//      interval, so every vertex gets the same name from its three arcs; the
//      conic (p, q) of the two smallest labels owns (emits) it.
// Lane order makes arcs and vertices come out in canonical order.  Then, per
// strut lane, the arcs of the strut are chained into its end loop ordered by
// the strut-frame angle phi (Sec. 4.3.1: arcs merged into an arc loop), and
// the circular arcs are grouped into hole contours (Sec. 5).  Subdivision
// uses Eq. 11 with step 2 pi / k and Eq. 12 sub-parameters; hole centres use
// Eq. 13.
//
// Precision: every node is first meshed in FP32.  A node goes to a second,
// FP64 pass of the same code when one of its vertices is ill-conditioned
// (the three surfaces meeting there have nearly dependent normals, so FP32
// rounding is amplified by the condition number kappa = |n1||n2||n3| /
// |det(n1, n2, n3)|) or when an FP32 consistency check fails.
#include <type_traits>

#include <utility>

#include "geom.h"

namespace lm {
namespace {

using namespace geo;

// ---------------------------------------------------------------------------
// per-node data in LDS

template <typename T>
struct ArcL {
    T o[3], a[3], b[3];
    T t1, t2;
    T dt;            // t2 - t1, kept with its own relative precision
    uint32_t ns, ne; // vertex names at t1 / t2
    int vs, ve;      // local vertex indices
    int p, q, full;
    int nseg, mbase, contour, fbase;
};

// Lanes per node and per-node capacities of one valence class: W lanes
// (64 / W nodes per wave), up to VM incident struts, AC arcs, VC vertices.
template <int VM_, int AC_, int VC_, int W_>
struct Cfg {
    static constexpr int VM = VM_, AC = AC_, VC = VC_, W = W_;
};
using CfgV4 = Cfg<4, 16, 16, 16>;   // v <= 4: four nodes per wave
using CfgV8 = Cfg<8, 32, 24, 32>;   // v <= 8: two nodes per wave
using CfgV16 = Cfg<kVmax, kAcap, kVcap, 64>;
// v = kVmax + 1 .. kVmaxBig: one node per block of kBigWaves waves, lanes of
// all its waves over the node's conics and samples, the node's data in the
// block's LDS (the paper's several warps per heavy workload, Sec. 4.3.3)
using CfgBig = Cfg<kVmaxBig, kAcapBig, kVcapBig, 64 * kBigWaves>;
// FP64 pass only: v = kVmax + 1 .. kVmaxMid on two waves
using CfgMid = Cfg<kVmaxMid, kAcapMid, kVcapMid, 128>;

template <typename T, typename C>
struct Shared {
    SL<T> S[C::VM + 1];
    ArcL<T> A[C::AC];
    uint32_t vname[C::VC];
    T vx[C::VC], vy[C::VC], vz[C::VC];
    uint8_t loop_arc[2 * C::AC];
    int8_t loop_dir[2 * C::AC];
    uint8_t loop_ord[2 * C::AC];
    int loop_base[C::VM + 2];
    int loop_len[C::VM + 1];  // samples |L_m|
    int loop_cnt[C::VM + 1];  // arcs per loop, then fill cursor
    int loop_first[C::VM + 1];
    int loop_full[C::VM + 1];
    uint16_t loop_next[2 * C::AC];
    int vdeg[C::VC];
    uint32_t clabel[C::AC];
    T hc[C::AC][3];           // hole centre (local) per contour
    int entry_off[2 * C::AC + 1];   // first loop sample of each loop entry
    uint8_t entry_m[2 * C::AC];     // strut label of each loop entry
    uint16_t entry_arc[2 * C::AC];  // arc of each loop entry | 0x8000 when run forward
    int loop_desc[C::VM + 1];       // descents of phi along each loop
    int loop_rot[C::VM + 1];        // loop position of the smallest phi
    T ph_first[C::VM + 1], ph_last[C::VM + 1];  // phi keys of each loop's ends
    int lbase[C::VM + 2];           // loop samples before each strut's loop
    uint8_t wmark[C::W <= 64 ? C::W : 1];  // loop entries starting in a window of samples
    int status, n_arc, n_vert, n_contour;
    int wsum, fsum, ncirc;
    int64_t rec;                    // first word of the node record, -1: none
};


__device__ inline uint32_t vname3(int a, int b, int c, int root)
{
    return ((uint32_t)a << 24) | ((uint32_t)b << 16) | ((uint32_t)c << 8) | (uint32_t)root;
}

// sorted triple of {p, q, r} (p < q already), branch free
struct Tri3 {
    int x, y, z;
};
__device__ inline Tri3 sort3(int p, int q, int r)
{
    const int x = min(p, r), z = max(q, r);
    return Tri3{x, p + q + r - x - z, z};
}

__device__ inline uint32_t tie_name(int p, int q, int r, int root)
{
    const Tri3 t = sort3(p, q, r);
    return vname3(t.x, t.y, t.z, root);
}

// Lane moves within a wave by DPP (gfx9 controls): row_shr:n shifts by n
// lanes within each row of 16, row_bcast:15 sends lane 15 of each row to the
// next row, row_bcast:31 sends lane 31 to rows 2 and 3, wave_shr:1 shifts the
// whole wave by one lane.  Lanes without a source, and rows left out by the
// row mask, read 0.  They run in the vector ALU, without the LDS round trip
// of a lane permute.
constexpr int kDppRowShr = 0x110, kDppWaveShr1 = 0x138, kDppBcast15 = 0x142, kDppBcast31 = 0x143;
template <int CTRL, int ROWS = 0xf>
__device__ inline int dpp_move(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWS, 0xf, true);
}

// inclusive scan over aligned groups of W = 16, 32 or 64 lanes of the wave:
// within rows, then the rows' totals carried forward
template <int W>
__device__ inline int wave_incl_scan(int x)
{
    x += dpp_move<kDppRowShr + 1>(x);
    x += dpp_move<kDppRowShr + 2>(x);
    x += dpp_move<kDppRowShr + 4>(x);
    x += dpp_move<kDppRowShr + 8>(x);
    if constexpr (W >= 32) x += dpp_move<kDppBcast15, 0xa>(x);
    if constexpr (W >= 64) x += dpp_move<kDppBcast31, 0xc>(x);
    return x;
}

// x of the last lane of the lane's group of W lanes (every lane of the wave
// holds a value)
template <int W>
__device__ inline int group_last_lane(int x)
{
    if constexpr (W == 64) {
        return __builtin_amdgcn_readlane(x, 63);
    } else {
        const int g = (int)(threadIdx.x & 63) / W;
        int r = __builtin_amdgcn_readlane(x, W - 1);
#pragma unroll
        for (int i = 1; i < 64 / W; ++i) {
            const int t = __builtin_amdgcn_readlane(x, i * W + W - 1);
            if (g == i) r = t;
        }
        return r;
    }
}

// exclusive scan over the W lanes of a node; every lane of the group must
// call it.  A group wider than a wave (the whole block) combines the waves'
// totals through LDS.
template <int W>
__device__ inline int group_excl_scan(int x, int *total)
{
    if constexpr (W == 1) {
        *total = x;
        return 0;
    } else if constexpr (W <= 64) {
        static_assert(W >= 16, "groups of 16, 32 or 64 lanes");
        const int inc = wave_incl_scan<W>(x);
        *total = group_last_lane<W>(inc);
        return inc - x;
    } else {
        __shared__ int s_part[W / 64];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int inc = wave_incl_scan<64>(x);
        if (lane == 63) s_part[wv] = inc;
        __syncthreads();
        int before = 0, tot = 0;
#pragma unroll
        for (int i = 0; i < W / 64; ++i) {
            const int pv = s_part[i];
            if (i < wv) before += pv;
            tot += pv;
        }
        __syncthreads();  // s_part is reused by the next call
        *total = tot;
        return before + inc - x;
    }
}

// x of lane 8 g + S in the lane's group g of 8 lanes (row_newbcast:n sends
// lane n of each row of 16 to the whole row)
template <int S>
__device__ inline int group8_lane(int x)
{
    const int a = __builtin_amdgcn_update_dpp(0, x, 0x150 + S, 0xf, 0xf, false);
    const int b = __builtin_amdgcn_update_dpp(0, x, 0x158 + S, 0xf, 0xf, false);
    return (threadIdx.x & 8) ? b : a;
}

template <int W>
__device__ inline void prev_last_bits(int x, int carry, int &prev, int &last)
{
    prev = dpp_move<kDppWaveShr1>(x);
    if ((threadIdx.x & (W - 1)) == 0) prev = carry;
    last = group_last_lane<W>(x);
}

// x of the previous lane of the group (lane 0: carry) and of its last lane
template <int W, typename T>
__device__ inline void group_prev_last(T x, T carry, T &prev, T &last)
{
    const int lane = threadIdx.x & (W - 1);
    if constexpr (W == 1) {
        prev = carry;
        last = x;
    } else if constexpr (W <= 64) {
        static_assert(W >= 16, "groups of 16, 32 or 64 lanes");
        if constexpr (sizeof(T) == 4) {
            int p, l;
            prev_last_bits<W>(__float_as_int(x), __float_as_int(carry), p, l);
            prev = __int_as_float(p);
            last = __int_as_float(l);
        } else {
            const int2 xv = *(const int2 *)&x, cv = *(const int2 *)&carry;
            int2 pv, lv;
            prev_last_bits<W>(xv.x, cv.x, pv.x, lv.x);
            prev_last_bits<W>(xv.y, cv.y, pv.y, lv.y);
            prev = *(const T *)&pv;
            last = *(const T *)&lv;
        }
    } else {
        __shared__ T s_x[W];
        s_x[lane] = x;
        __syncthreads();
        prev = lane ? s_x[lane - 1] : carry;
        last = s_x[W - 1];
        __syncthreads();
    }
}

// 64-bit x moved like dpp_move (both halves)
template <int CTRL, int ROWS = 0xf>
__device__ inline uint64_t dpp_move64(uint64_t x)
{
    const uint32_t lo = (uint32_t)dpp_move<CTRL, ROWS>((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)dpp_move<CTRL, ROWS>((int)(uint32_t)(x >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// sum modulo 2^64 over the W lanes of a node (every lane gets it): an
// inclusive DPP scan, then the group's last lane; a group wider than a wave
// adds the waves' sums through LDS
template <int W>
__device__ inline uint64_t group_sum_u64(uint64_t x)
{
    if constexpr (W == 1) {
        return x;
    } else if constexpr (W <= 64) {
        static_assert(W >= 16, "groups of 16, 32 or 64 lanes");
        x += dpp_move64<kDppRowShr + 1>(x);
        x += dpp_move64<kDppRowShr + 2>(x);
        x += dpp_move64<kDppRowShr + 4>(x);
        x += dpp_move64<kDppRowShr + 8>(x);
        if constexpr (W >= 32) x += dpp_move64<kDppBcast15, 0xa>(x);
        if constexpr (W >= 64) x += dpp_move64<kDppBcast31, 0xc>(x);
        const uint32_t lo = (uint32_t)group_last_lane<W>((int)(uint32_t)x);
        const uint32_t hi = (uint32_t)group_last_lane<W>((int)(uint32_t)(x >> 32));
        return (uint64_t)lo | ((uint64_t)hi << 32);
    } else {
        __shared__ uint64_t s_part[W / 64];
        x = group_sum_u64<64>(x);
        if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = x;
        __syncthreads();
        uint64_t t = 0;
#pragma unroll
        for (int i = 0; i < W / 64; ++i) t += s_part[i];
        __syncthreads();
        return t;
    }
}

// The node's status word as every lane of the group sees it at this point.
// Within a wave the lanes read it together; a group of several waves reads
// it between two barriers, so that no wave can already be setting bits of
// the next phase while another still reads (all lanes take the same branch).
template <int W, typename SH>
__device__ inline int group_status(SH &sh)
{
    if constexpr (W <= 64) {
        return sh.status;
    } else {
        __syncthreads();
        const int s = sh.status;
        __syncthreads();
        return s;
    }
}

// f(i) for i = lo + lane, lo + lane + W, ... up to hi (inclusive; hi is at
// most the valence + 1): one test when a node has more lanes than that, a
// loop otherwise (one lane per node)
template <int W, int VM, typename F>
__device__ inline void over_lanes(int lane, int lo, int hi, F &&f)
{
    if constexpr (W > VM + 1) {
        if (lo + lane <= hi) f(lo + lane);
    } else {
        for (int i = lo + lane; i <= hi; i += W) f(i);
    }
}

// ---------------------------------------------------------------------------
// trimming of one conic: intersection of circular intervals

// Pseudo-angle of the direction (sin t, cos t) ~ (s, c): a value in [0, 4)
// that increases with t in [0, 2 pi) (a half turn adds exactly 2), computed
// with one division instead of an arctangent.  Interval bookkeeping on the
// circle only compares and adds such values, so it runs in this measure.
template <typename T>
__device__ inline T pang(T s, T c)
{
    const T u = m_qdiv(c, m_abs(s) + m_abs(c));
    T p = s >= (T)0 ? (T)1 - u : (T)3 + u;
    return p >= (T)4 ? (T)0 : p;
}

// kept arcs per conic: 2 in FP32 (a third sends the node to FP64), 4 in FP64
template <typename T>
struct NPieces {
    static constexpr int n = sizeof(T) == 4 ? 2 : kPieces;
};

template <typename T>
struct Pc {
    T s, len;  // pseudo-angle of the start, pseudo length
    int rs, re;  // constraints whose lower / upper end bound the piece
};

// A kept piece in final form.
template <typename T>
struct Piece {
    T ss, sc, es, ec;  // directions (sin t, cos t) of the ends, unnormalised
    T len;
    int rs, re;
    int roots;  // bit 0: root of the start tie, bit 1: root of the end tie
};

template <typename T>
struct TrimOut {
    int n;        // arcs
    int full;     // whole conic kept
    int ovf;      // too many pieces
    Piece<T> pc[NPieces<T>::n];
};

// Constraint r on conic (p, q): P_p - P_r = A sin t + B cos t + Cc.  Keeping
// P_p >= P_r is R cos(t - psi) >= -Cc with psi = atan2(A, B) (Eqs. 8-9),
// i.e. t - psi in [-beta, beta] with cos beta = -Cc / R.
template <typename T>
struct Cons {
    T A, B, Cc, R;
};

template <typename T>
__device__ inline Cons<T> cons_of(const SL<T> *S, V3<T> gp, T hp, int r, const Con<T> &C)
{
    V3<T> gr = r ? gvec(S[r]) : zero3<T>();
    T hr = r ? S[r].h : (T)0;
    V3<T> dg = gp - gr;
    Cons<T> k;
    k.A = dot(dg, C.a);
    k.B = dot(dg, C.b);
    k.Cc = dot(dg, C.o) - (hp - hr);
    k.R = m_sqrt(k.A * k.A + k.B * k.B);
    return k;
}

// Directions of the kept interval's ends: (A, B) / R turned by -beta (lo)
// and +beta (hi), scaled by R^2.
template <typename T>
__device__ inline void cons_ends(const Cons<T> &k, T &los, T &loc, T &his, T &hic)
{
    const T Sn = m_sqrt((k.R - k.Cc) * (k.R + k.Cc));  // R sin(beta)
    los = -k.A * k.Cc - k.B * Sn;
    loc = -k.B * k.Cc + k.A * Sn;
    his = -k.A * k.Cc + k.B * Sn;
    hic = -k.B * k.Cc - k.A * Sn;
}

// Rank (0/1) of the upper end of constraint r's interval among the two tie
// points of (p, q, r) along d = (g_x - g_y) x (g_x - g_z), (x, y, z) =
// sorted (p, q, r): the chord x(hi) - x(lo) is parallel to the tie line and
// to a B - b A.
template <typename T>
__device__ inline int hi_root(const SL<T> *S, int p, int q, int r, const Con<T> &C, const Cons<T> &k)
{
    const Tri3 xyz = sort3(p, q, r);
    V3<T> gx = xyz.x ? gvec(S[xyz.x]) : zero3<T>();
    V3<T> d = cross(gx - gvec(S[xyz.y]), gx - gvec(S[xyz.z]));
    return dot(C.a * k.B - C.b * k.A, d) > (T)0 ? 1 : 0;
}

// Kept set of constraint r on conic (p, q): 0 never active, 1 removes the
// whole conic, 2 the interval [lo, lo + lc] in pseudo-angle.
template <typename T>
__device__ inline int cons_interval(const SL<T> *S, V3<T> gp, T hp, int r, const Con<T> &C, T &lo, T &lc)
{
    const T tp = (T)4;  // full turn in pseudo-angle
    const Cons<T> k = cons_of(S, gp, hp, r, C);
    if (k.Cc >= k.R) return 0;   // never active
    if (k.Cc <= -k.R) return 1;  // removes the whole conic
    T los, loc, his, hic;
    cons_ends(k, los, loc, his, hic);
    lo = pang(los, loc);
    const T hi = pang(his, hic);
    lc = hi - lo;
    if (lc < (T)0) lc += tp;
    // more than a half turn exactly when Cc > 0: a kept interval that
    // comes out almost empty although Cc > 0 is almost the whole turn
    // (its gap is below rounding), one that comes out almost whole
    // although Cc < 0 is almost empty.  Near a half turn (Cc near 0)
    // the computed length stands.
    if (k.Cc > (T)0 && lc < (T)1) return 0;
    if (k.Cc < (T)0 && lc > (T)3) return 1;
    return 2;
}

// Running intersection of the kept sets of a conic, taken in constraint
// order.
template <typename T>
struct TrimRun {
    Pc<T> pc[NPieces<T>::n];
    int n = 1, full = 1;
    bool ovf = false, done = false;
};

template <typename T>
__device__ inline void trim_step(TrimRun<T> &st, int kind, T lo, T lc, int r)
{
    constexpr int NP = NPieces<T>::n;
    const T tp = (T)4;
    if (st.done || kind == 0) return;
    if (kind == 1) {
        st.n = 0;
        st.full = 0;
        st.done = true;
        return;
    }
    if (st.full) {
        st.pc[0] = Pc<T>{lo, lc, r, r};
        st.n = 1;
        st.full = 0;
        return;
    }
    // intersect the current pieces with [lo, lo + lc]
    Pc<T> out[NP];
    int no = 0;
    auto push = [&](T s0, T l0, int rs, int re) {
#pragma unroll
        for (int j = 0; j < NP; ++j)
            if (j == no) out[j] = Pc<T>{s0, l0, rs, re};
        if (no < NP) ++no;
        else st.ovf = true;
    };
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        if (i < st.n) {
            const Pc<T> Pp = st.pc[i];
            T c0 = lo - Pp.s;
            if (c0 < (T)0) c0 += tp;
            const T c1 = c0 + lc;
            if (c0 < Pp.len) {
                const bool ns = c0 > (T)0, ne = c1 < Pp.len;
                push(ns ? lo : Pp.s, (ne ? c1 : Pp.len) - c0, ns ? r : Pp.rs, ne ? r : Pp.re);
            }
            if (c1 > tp) {
                const T w1 = c1 - tp;
                const bool ne = w1 < Pp.len;
                push(Pp.s, ne ? w1 : Pp.len, Pp.rs, ne ? r : Pp.re);
            }
        }
    }
    st.n = no;
#pragma unroll
    for (int j = 0; j < NP; ++j) st.pc[j] = out[j];
    if (no == 0) st.done = true;
}

// Split trimming round: the constraint of lane S of the group (kind, label,
// interval) intersected in constraint order, S = 0 .. 6
template <int... S>
__device__ inline void split_steps(TrimRun<float> &st, int kind, int r, float lo, float lc,
                                   std::integer_sequence<int, S...>)
{
    (trim_step(st, group8_lane<S>(kind), __int_as_float(group8_lane<S>(__float_as_int(lo))),
               __int_as_float(group8_lane<S>(__float_as_int(lc))), group8_lane<S>(r)),
     ...);
}

// final form: end directions and tie roots of every piece
template <typename T>
__device__ inline void trim_finish(const SL<T> *S, int p, int q, const Con<T> &C, V3<T> gp, T hp,
                                   const TrimRun<T> &st, TrimOut<T> &TR)
{
    constexpr int NP = NPieces<T>::n;
    TR.n = st.n;
    TR.full = st.full;
    TR.ovf = st.ovf ? 1 : 0;
    if (st.full) return;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        if (i < st.n) {
            Piece<T> &o = TR.pc[i];
            T a0, a1, a2, a3;
            const Cons<T> ks = cons_of(S, gp, hp, st.pc[i].rs, C);
            cons_ends(ks, o.ss, o.sc, a2, a3);
            const int root_s = 1 - hi_root(S, p, q, st.pc[i].rs, C, ks);
            const Cons<T> ke = cons_of(S, gp, hp, st.pc[i].re, C);
            cons_ends(ke, a0, a1, o.es, o.ec);
            const int root_e = hi_root(S, p, q, st.pc[i].re, C, ke);
            o.len = st.pc[i].len;
            o.rs = st.pc[i].rs;
            o.re = st.pc[i].re;
            o.roots = root_s | (root_e << 1);
        }
    }
}

template <typename T>
__device__ void trim_conic(const SL<T> *S, int v, int p, int q, const Con<T> &C, TrimOut<T> &TR)
{
    const V3<T> gp = p ? gvec(S[p]) : zero3<T>();
    const T hp = p ? S[p].h : (T)0;
    TrimRun<T> st;
    for (int r = 0; r <= v; ++r) {
        if (r == p || r == q) continue;
        T lo = (T)0, lc = (T)0;
        const int kind = cons_interval(S, gp, hp, r, C, lo, lc);
        trim_step(st, kind, lo, lc, r);
        if (st.done) break;
    }
    trim_finish(S, p, q, C, gp, hp, st, TR);
}

// Conic point at the direction (sin t, cos t) ~ (s, c)
template <typename T>
__device__ inline V3<T> conic_dir(const Con<T> &C, T s, T c)
{
    const T inv = (T)1 / m_sqrt(s * s + c * c);
    return C.o + C.a * (s * inv) + C.b * (c * inv);
}

// Parameter range [t1, t2] (t1 in [0, 2 pi)) and span of a kept piece
template <typename T>
__device__ inline void piece_range(const Piece<T> &pc, T &t1, T &t2, T &dt)
{
    const T tp = Cst<T>::two_pi;
    T ts = m_atan2(pc.ss, pc.sc), te = m_atan2(pc.es, pc.ec);
    if (ts < (T)0) ts += tp;
    if (te < (T)0) te += tp;
    T span = te - ts;
    if (span < (T)0) span += tp;
    // agree with the pseudo length where rounding puts the ends of an
    // almost empty or almost full piece on the wrong side of each other
    if (pc.len < (T)1 && span > (T)1.5 * Cst<T>::pi) span = (T)0;
    if (pc.len > (T)3 && span < (T)0.5 * Cst<T>::pi) span = tp;
    t1 = ts;
    t2 = ts + span;
    dt = span;
}

// Whether FP32 can be trusted with the tie point w of labels p < q < r.  The
// three surfaces through it are cone p (normal n1 = w - P_p g_p, or w for the
// sphere) and the planes P_p = P_q, P_p = P_r (normals n2 = g_p - g_q,
// n3 = g_p - g_r).  Not trusted when
//   - the condition number |n1||n2||n3| / |det(n1, n2, n3)| exceeds
//     kappa_max (FP32 rounding of the surfaces is amplified that much), or
//   - the FP32 error of the point as the solution of the tie equations
//     exceeds kVertexErr rho: the equations' residuals carry rounding of
//     the size of their terms (|g||w| for the planes, |w|^2 + P_p^2 + rho^2
//     for the cone), mapped through the inverse Jacobian (cofactors over
//     the determinant).  The condition number alone misses points far from
//     the node centre on the seams of nearly parallel struts.
template <typename T>
__device__ inline bool tie_trusted(const SL<T> *S, int p, int q, int r, V3<T> w, T rho, T kappa_max)
{
    const V3<T> gp = p ? gvec(S[p]) : zero3<T>();
    const T pp = p ? dot(gp, w) - S[p].h : (T)0;
    const V3<T> gq = gvec(S[q]), gr = r ? gvec(S[r]) : zero3<T>();
    const V3<T> n1 = w - gp * pp, n2 = gp - gq, n3 = gp - gr;
    const V3<T> c12 = cross(n1, n2), c23 = cross(n2, n3), c31 = cross(n3, n1);
    const T det = m_abs(dot(n1, c23));
    if (!(det > (T)0)) return false;
    if (m_sqrt(dot(n1, n1) * dot(n2, n2) * dot(n3, n3)) > kappa_max * det) return false;
    const T lw = m_sqrt(dot(w, w));
    const T lgp = m_sqrt(dot(gp, gp)), lq = m_sqrt(dot(gq, gq)), lr = m_sqrt(dot(gr, gr));
    const T bound = m_sqrt(dot(c31, c31)) * ((T)2 * (lgp + lq) * lw) +
                    m_sqrt(dot(c12, c12)) * ((T)2 * (lgp + lr) * lw) +
                    m_sqrt(dot(c23, c23)) * (lw * lw + pp * pp + rho * rho);
    return !(bound * (T)kFp32Eps > (T)(2.0f * kVertexErr) * rho * det);
}

// ---------------------------------------------------------------------------

// Ordering key of the strut angle phi = atan2(y, x): a pseudo-angle in
// (-2, 2] (a half turn is 2), increasing with phi in (-pi, pi].  The band
// zipper only compares angles about one strut axis, so it uses this key.
template <typename T>
__device__ inline T phi_key(T y, T x)
{
    const T u = m_qdiv(x, m_abs(y) + m_abs(x));
    return y >= (T)0 ? (T)1 - u : u - (T)1;
}

template <typename T>
__device__ inline Con<T> arc_con(const ArcL<T> &A)
{
    Con<T> C;
    C.o = v3(A.o[0], A.o[1], A.o[2]);
    C.a = v3(A.a[0], A.a[1], A.a[2]);
    C.b = v3(A.b[0], A.b[1], A.b[2]);
    return C;
}

template <typename SH>
__device__ inline int find_vert(const SH &sh, uint32_t name)
{
    int lo = 0, hi = sh.n_vert - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        uint32_t m = sh.vname[mid];
        if (m == name) return mid;
        if (m < name) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// Eq. 12 index ii (1..nseg-1) of an interior point -> node-local mesh index
template <typename T>
__device__ inline int interior_idx(const ArcL<T> &A, int ii)
{
    bool fwd = A.full || A.ns <= A.ne;
    return A.mbase + (fwd ? ii - 1 : A.nseg - 1 - ii);
}

template <typename T>
__device__ inline T sub_param(const ArcL<T> &A, int ii)
{
    return A.t1 + A.dt * (T)ii / (T)A.nseg;
}

template <typename T, typename C>
__device__ inline V3<T> vert_pos(const Shared<T, C> &sh, int i) { return v3(sh.vx[i], sh.vy[i], sh.vz[i]); }

// Eq. 12 point ii of arc A: the formula of arc_point_f32 (whole conics
// directly, arcs from their start vertex with the differences in product
// form), in the node's precision
template <typename T, typename C>
__device__ inline V3<T> interior_pt(const Shared<T, C> &sh, const ArcL<T> &A, int ii)
{
    if constexpr (sizeof(T) == 4) {
        const float x1[3] = {A.full ? 0.f : sh.vx[A.vs], A.full ? 0.f : sh.vy[A.vs], A.full ? 0.f : sh.vz[A.vs]};
        const float3 w = arc_point_f32(A.o, A.a, A.b, x1, A.t1, A.dt, ii, A.nseg, A.full != 0);
        return v3(w.x, w.y, w.z);
    } else {
        if (A.full) return conic_at(arc_con(A), sub_param(A, ii));
        const T h = (T)0.5 * A.dt * (T)ii / (T)A.nseg;
        T sh_, ch_, sm, cm;
        m_sincos(h, &sh_, &ch_);
        m_sincos(A.t1 + h, &sm, &cm);
        const T ds = (T)2 * cm * sh_, dc = (T)-2 * sm * sh_;
        const Con<T> Cn = arc_con(A);
        return vert_pos(sh, A.vs) + Cn.a * ds + Cn.b * dc;
    }
}

struct Params {
    Inputs in;
    Work w;
    int k;
    float kappa_max;  // FP32 nodes with a vertex above this go to FP64
    // re-subdivision: the meta-mesh comes from these records instead
    const uint32_t *src_rec;
    const int64_t *src_node_rec;
    // nodes to solve in full after a re-subdivision pass: per class a list
    // at the class's queue offset, its length and a work counter
    int32_t *redo;
    int32_t *redo_cnt;  // [4]
    int32_t *redo_ctr;  // [4]
    // sink mode: where the counts and hashes of vertices and fans go
    SinkOut sink;
};

// statuses that FP64 may resolve
constexpr int kRetry = NS_NON_ELLIPTIC | NS_LOOP | NS_TOPOLOGY | NS_PREC | NS_CAPACITY;

// The whole per-node computation: counts, and the node record for the
// expansion pass.
// Subdivision at resolution k and the node record, for a node whose
// meta-mesh (arcs, vertices, end loops, contours) is in LDS with its status.
// Sink mode: counts and hashes of the node's mesh vertices (meta-vertices,
// Eq. 12 interior points, Eq. 13 hole centres, in the stored mode's node-local
// numbering and FP32 positions) and of its hole fans, added to the node's
// chunk or part.  The Eq. 12 points arrive already summed (hv, sx, sy, sz) by
// the loop walk, which evaluates them anyway.
template <typename T, typename CF>
__device__ __forceinline__ void sink_hash_node(const Params &P, Shared<T, CF> &sh, const int64_t n, const int M,
                                               const int F, uint64_t hv, uint64_t sx, uint64_t sy, uint64_t sz)
{
    constexpr int WL = CF::W;
    const int lane = threadIdx.x & (WL - 1);
    const SinkOut &S = P.sink;
    const float4 c4 = P.w.node4[n];
    const int64_t ln = sink_local_node(S, n);
    const int V = sh.n_vert, wsum = sh.wsum, ncirc = sh.ncirc;
    uint64_t ht = 0;
    // meta-vertices (local indices 0 .. V-1) and hole centres (wsum .. M-1);
    // the Eq. 12 points between them came in with hv, sx, sy, sz
    for (int t = lane; t < V + (M - wsum); t += WL) {
        const int i = t < V ? t : wsum + (t - V);
        float3 w;
        if (i < V) {
            w = make_float3((float)sh.vx[i], (float)sh.vy[i], (float)sh.vz[i]);
        } else {
            const int c = i - wsum;
            w = make_float3((float)sh.hc[c][0], (float)sh.hc[c][1], (float)sh.hc[c][2]);
        }
        const float x = c4.x + w.x, y = c4.y + w.y, z = c4.z + w.z;
        hv += vert_key(vid_of(ln, i), x, y, z);
        sx += (uint64_t)llrint((double)x * 1048576.0);
        sy += (uint64_t)llrint((double)y * 1048576.0);
        sz += (uint64_t)llrint((double)z * 1048576.0);
    }
    // hole fans: one triangle per circular-arc segment, apex at the contour's
    // hole centre, oriented outward
    for (int i = lane; i < F; i += WL) {
        int lo = 0, hi = ncirc - 1;  // last circular arc with fbase <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sh.A[mid].fbase <= i) lo = mid;
            else hi = mid - 1;
        }
        const ArcL<T> &A = sh.A[lo];
        const bool fwd = A.full || A.ns <= A.ne, lower = sh.S[A.q].lower;
        const int nseg = A.nseg, sseg = i - A.fbase;
        const int i0 = fwd ? sseg : nseg - sseg, i1 = fwd ? sseg + 1 : nseg - sseg - 1;
        const int lo_i = i0 < i1 ? i0 : i1, hi_i = i0 < i1 ? i1 : i0;
        const int u = lo_i == 0 ? A.vs : A.mbase + (fwd ? lo_i - 1 : nseg - 1 - lo_i);
        const int u2 = hi_i == nseg ? A.ve : A.mbase + (fwd ? hi_i - 1 : nseg - 1 - hi_i);
        ht += tri_key(vid_of(ln, wsum + A.contour), vid_of(ln, lower ? u2 : u), vid_of(ln, lower ? u : u2));
    }
    hv = group_sum_u64<WL>(hv);
    sx = group_sum_u64<WL>(sx);
    sy = group_sum_u64<WL>(sy);
    sz = group_sum_u64<WL>(sz);
    ht = group_sum_u64<WL>(ht);
    if (lane == 0) {
        const int32_t part = S.node_part ? S.node_part[n] : 0;
        sink_add(S, part, 0, (uint64_t)F);
        sink_add(S, part, 1, ht);
        sink_add(S, part, 2, (uint64_t)M);
        sink_add(S, part, 3, hv);
        sink_add(S, part, 4, sx);
        sink_add(S, part, 5, sy);
        sink_add(S, part, 6, sz);
    }
}

// SINK: instead of a node record for the expansion and the bands, only the
// strut end loops are kept (for the bands); the node's mesh vertices and hole
// fans are counted and hashed here (sink mode).
template <typename T, typename CF, bool SINK>
__device__ __forceinline__ void node_tail(const Params &P, Shared<T, CF> &sh, const int64_t n, const int k, const int v,
                          const int64_t row, const T rho, const V3<T> cen)
{
    constexpr int WL = CF::W;
    constexpr bool F32 = sizeof(T) == 4;
    // arc indices above 127 or loop positions above 255 need 16-bit entries
    // in the record's loop table
    constexpr bool WIDE = CF::AC > 127;
    const T tp = Cst<T>::two_pi;
    const int lane = threadIdx.x & (WL - 1);
    const Work &W = P.w;
    const int64_t N = P.in.n_nodes;
    (void)tp;
    (void)cen;
    (void)k;
    // sink mode: the node's Eq. 12 points are hashed where the loop walk
    // evaluates them (each once, on the loop of its arc's label q), for
    // nodes of the hashed range
    uint64_t pt_v = 0, pt_x = 0, pt_y = 0, pt_z = 0;
    const bool hash_pts = SINK && n >= P.sink.n0 && n < P.sink.n1;
    const int64_t ln_sink = SINK ? sink_local_node(P.sink, n) : 0;
    if (group_status<WL>(sh)) goto finish;

    // ---- mesh-vertex layout, hole centres, loop phi check -------------------
    {
        const int E = sh.n_arc, V = sh.n_vert, NC = sh.n_contour;
        // prefix sums over the arcs (lanes in chunks, carried): interior
        // points of each arc, and fan triangles of the circular arcs (which
        // sort first; one fan triangle per segment)
        {
            int mb = V, fb = 0, nc = 0;
            for (int j0 = 0; j0 < E; j0 += WL) {
                const int j = j0 + lane;
                int ni = 0, nf = 0, ic = 0;
                if (j < E) {
                    const ArcL<T> &A = sh.A[j];
                    ni = A.nseg - 1;
                    if (A.p == 0) {
                        nf = A.nseg;
                        ic = 1;
                    }
                }
                int ti, tf, tc;
                const int ei = group_excl_scan<WL>(ni, &ti), ef = group_excl_scan<WL>(nf, &tf);
                group_excl_scan<WL>(ic, &tc);
                if (j < E) {
                    sh.A[j].mbase = mb + ei;
                    sh.A[j].fbase = fb + ef;
                }
                mb += ti;
                fb += tf;
                nc += tc;
            }
            if (lane == 0) {
                sh.wsum = mb;  // first hole-centre index
                sh.fsum = fb;
                sh.ncirc = nc;
            }
        }
        __syncthreads();
        // Eq. 13: barycentre of each contour's vertices (each once: half of
        // both ends of every arc plus its interior points), projected on the
        // nodal sphere; the point opposite is used when the projection falls
        // under a strut, and -sum(e_m) when the barycentre is within 1e-3 rho
        // of the centre.
        for (int c = lane; c < NC; c += WL) {
            V3<T> sum = zero3<T>();
            int cntv = 0;
            for (int j = 0; j < E && sh.A[j].p == 0; ++j) {
                const ArcL<T> &A = sh.A[j];
                if (A.contour != c) continue;
                sum = sum + (vert_pos(sh, A.vs) + vert_pos(sh, A.ve)) * (T)0.5;
                for (int ii = 1; ii < A.nseg; ++ii) sum = sum + interior_pt(sh, A, ii);
                cntv += A.nseg;
            }
            V3<T> b = sum * ((T)1 / (T)cntv);
            T bl = m_sqrt(dot(b, b));
            // the apex direction b/|b| amplifies rounding by rho/|b|; the
            // fallback decision near |b| = 1e-3 rho is fragile as well
            if (F32 && bl * (T)P.kappa_max < rho) atomicOr(&sh.status, NS_PREC);
            V3<T> dir;
            if (bl >= (T)1e-3 * rho) {
                dir = b * ((T)1 / bl);
            } else {
                V3<T> se = zero3<T>();
                for (int m = 1; m <= v; ++m) se = se + v3(sh.S[m].ex, sh.S[m].ey, sh.S[m].ez);
                T sl = m_sqrt(dot(se, se));
                if (sl < (T)1e-3) { atomicOr(&sh.status, NS_TOPOLOGY); sl = (T)1; }
                dir = se * ((T)-1 / sl);
            }
            for (int flip = 0; flip < 2; ++flip) {
                T pm = (T)-1e30;
                for (int m = 1; m <= v; ++m) pm = m_max(pm, dot(gvec(sh.S[m]), dir * rho) - sh.S[m].h);
                if (pm <= (T)0) break;
                if (flip) atomicOr(&sh.status, NS_TOPOLOGY);
                dir = dir * (T)-1;
            }
            sh.hc[c][0] = dir.x * rho;
            sh.hc[c][1] = dir.y * rho;
            sh.hc[c][2] = dir.z * rho;
        }
        __syncthreads();
        if (group_status<WL>(sh)) goto finish;
        // strut end loops must be graphs over phi: every step (mod 2 pi)
        // positive and exactly one descent, i.e. one turn.  Lanes run over
        // all loop samples of the node and store them in the node record.
        // loop entries (arcs of every loop, loops in label order): first
        // sample of each entry by a carried prefix sum over the lanes
        {
            const int nent = sh.loop_base[v + 1];
            int off = 0;
            for (int e0 = 0; e0 < nent; e0 += WL) {
                const int e = e0 + lane;
                int ns = 0, m = 1;
                if (e < nent) {
                    while (sh.loop_base[m + 1] <= e) ++m;
                    const int pp = sh.loop_base[m] + sh.loop_ord[e];
                    const int aj = sh.loop_arc[pp];
                    ns = sh.A[aj].nseg;
                    sh.entry_arc[e] = (uint16_t)(aj | (sh.loop_dir[pp] > 0 ? 0x8000 : 0));
                }
                int tot;
                const int ex = group_excl_scan<WL>(ns, &tot);
                if (e < nent) {
                    sh.entry_off[e] = off + ex;
                    sh.entry_m[e] = (uint8_t)m;
                }
                off += tot;
            }
            if (lane == 0) sh.entry_off[nent] = off;
        }
        __syncthreads();
        // index v: the total
        over_lanes<WL, CF::VM>(lane, 0, v, [&](int l) { sh.lbase[l + 1] = sh.entry_off[sh.loop_base[l + 1]]; });
        if (lane == 0) {
            const int off = sh.entry_off[sh.loop_base[v + 1]];
            // record space: bump allocation in the node's region
            // the node's interior points follow its hole centres
            const int HX = NC + sh.wsum - V;
            const int64_t words =
                (SINK ? 0 : rec_loop_word(V, E, HX, rec_table_bytes(v, sh.loop_base[v + 1], WIDE))) +
                (((int64_t)2 * off + 3) & ~(int64_t)3);
            const int g = (int)(n & (kRecRegions - 1));
            const int64_t region = W.rec_words / kRecRegions;
            const unsigned long long old = atomicAdd(&W.rec_top[g], (unsigned long long)words);
            if ((int64_t)old + words <= region) {
                sh.rec = (int64_t)g * region + (int64_t)old;
            } else {
                sh.rec = -1;
                atomicOr(&W.flags[0], DF_RECCAP);
            }
        }
        over_lanes<WL, CF::VM>(lane, 0, v - 1, [&](int l) {
            sh.loop_desc[l + 1] = 0;
            sh.loop_rot[l + 1] = 0;
        });
        __syncthreads();
        {
            const int nent = sh.loop_base[v + 1];
            const int ns_tot = sh.entry_off[nent];
            const int HX = NC + sh.wsum - V;
            int2 *rl = sh.rec >= 0
                           ? (int2 *)(W.rec + sh.rec + (SINK ? 0 : rec_loop_word(V, E, HX, rec_table_bytes(v, nent, WIDE))))
                           : nullptr;
            // the node's Eq. 12 points in the record (stored mode), indexed
            // by node-local mesh index: the expansion copies them
            uint32_t *RI = (!SINK && sh.rec >= 0) ? W.rec + sh.rec + rec_table_word(V, E, NC) - 3 * V : nullptr;
            // phi key and local mesh index of sample j of loop entry e (on
            // the loop of strut m); an interior point is stored by the loop
            // of its arc's label q (every arc is on that loop)
            auto sample = [&](int e, int m, int j, int &li) -> T {
                const uint32_t ea = sh.entry_arc[e];
                const ArcL<T> &A = sh.A[ea & 0x7fffu];
                const bool fw = (ea & 0x8000u) != 0;
                const int ii = fw ? j : A.nseg - j;
                li = j == 0 ? (fw ? A.vs : A.ve) : interior_idx(A, ii);
                const V3<T> w = j == 0 ? vert_pos(sh, li) : interior_pt(sh, A, ii);
                if (j != 0 && m == A.q) {
                    if (RI) {
                        RI[3 * li] = __float_as_uint((float)w.x);
                        RI[3 * li + 1] = __float_as_uint((float)w.y);
                        RI[3 * li + 2] = __float_as_uint((float)w.z);
                    }
                    if (hash_pts) {
                        // as stored: the point rounded once, plus the centre
                        const float x = (float)cen.x + (float)w.x, y = (float)cen.y + (float)w.y,
                                    z = (float)cen.z + (float)w.z;
                        pt_v += vert_key(vid_of(ln_sink, li), x, y, z);
                        pt_x += (uint64_t)llrint((double)x * 1048576.0);
                        pt_y += (uint64_t)llrint((double)y * 1048576.0);
                        pt_z += (uint64_t)llrint((double)z * 1048576.0);
                    }
                }
                // tangency circles are parametrised in the strut frame: phi
                // is the parameter itself
                if (A.p == 0) {
                    T st, ct;
                    m_sincos(sub_param(A, ii), &st, &ct);
                    return phi_key(st, ct);
                }
                const SL<T> &sm = sh.S[m];
                return phi_key(dot(w, v3(sm.qx, sm.qy, sm.qz)), dot(w, v3(sm.rx, sm.ry, sm.rz)));
            };
            // each lane checks the step from the previous sample of its loop
            // (the previous lane's, or the last of the previous chunk); the
            // step that closes a loop is checked afterwards.  A valid loop
            // has exactly one descent, just before its smallest phi.
            T carry = (T)0;
            int e_carry = -1;  // loop entry of the sample before the window
            for (int base = 0; base < ns_tot; base += WL) {
                const int sidx = base + lane;
                const bool act = sidx < ns_tot;
                int m = 1, idx = 0, nloop = 1, li = 0;
                T ph = (T)0;
                int e = 0;  // loop entry of sample sidx
                if constexpr (WL >= 16 && WL <= 64) {
                    // the entries that start in the window [base, base + WL)
                    // are e_carry + 1, e_carry + 2, ... (every entry has a
                    // sample): each marks its first sample, and a scan of the
                    // marks over the lanes gives every sample its entry
                    sh.wmark[lane] = 0;
                    const int ec = e_carry + 1 + lane;
                    if (ec < nent) {
                        const int o = sh.entry_off[ec] - base;
                        if (o < WL) sh.wmark[o] = 1;
                    }
                    __syncthreads();
                    e = e_carry + wave_incl_scan<WL>((int)sh.wmark[lane]);
                    e_carry = group_last_lane<WL>(e);
                } else if (act) {
                    int lo = 0, hi = nent - 1;  // last entry with entry_off <= sidx
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (sh.entry_off[mid] <= sidx) lo = mid;
                        else hi = mid - 1;
                    }
                    e = lo;
                }
                if (act) {
                    m = sh.entry_m[e];
                    idx = sidx - sh.lbase[m];
                    nloop = sh.loop_len[m];
                    ph = sample(e, m, sidx - sh.entry_off[e], li);
                }
                T prev, last;
                group_prev_last<WL>(ph, carry, prev, last);
                carry = last;
                if (act) {
                    if (idx == 0) {
                        sh.ph_first[m] = ph;
                    } else {
                        T dp = ph - prev;  // in key units: a full turn is 4
                        if (dp <= (T)-2) dp += (T)4;
                        if (dp > (T)2) dp -= (T)4;
                        if (!(dp > (T)0)) atomicOr(&sh.status, NS_LOOP);
                        if (ph < prev) {
                            atomicAdd(&sh.loop_desc[m], 1);
                            sh.loop_rot[m] = idx;
                        }
                    }
                    if (idx == nloop - 1) sh.ph_last[m] = ph;
                    if (rl) rl[sidx] = make_int2(li, __float_as_int((float)ph));
                }
            }
        }
        __syncthreads();
        over_lanes<WL, CF::VM>(lane, 0, v - 1, [&](int l) {
            const int m = l + 1;
            const T a = sh.ph_last[m], b = sh.ph_first[m];
            T dp = b - a;
            if (dp <= (T)-2) dp += (T)4;
            if (dp > (T)2) dp -= (T)4;
            if (!(dp > (T)0)) atomicOr(&sh.status, NS_LOOP);
            if (b < a) {
                atomicAdd(&sh.loop_desc[m], 1);
                sh.loop_rot[m] = 0;
            }
        });
        __syncthreads();
        over_lanes<WL, CF::VM>(lane, 0, v - 1, [&](int l) {
            if (sh.loop_desc[l + 1] != 1) atomicOr(&sh.status, NS_LOOP);
            W.he_rot[row + l] = sh.loop_rot[l + 1];
        });
        __syncthreads();
    }

finish:
    __syncthreads();
    {
        const int status = sh.status;
        const int E = sh.n_arc, V = sh.n_vert, NC = sh.n_contour;
        if (status) {
            if (lane == 0) {
                for (int c = 0; c < kNodeCols; ++c) W.node_cnt[c * N + n] = 0;
                W.node_cnt[NC_STATUS * N + n] = status & ~NS_PREC;
                W.node_rec[n] = -1;
                // hand the node to the FP64 pass when precision may be at fault
                const bool retry = F32 && (status & kRetry);
                if (retry) W.fb_list[atomicAdd(&W.flags[2], 1)] = (int32_t)n;
                // FP64, two-wave class: a node beyond its capacities goes on
                // to the four-wave kernel (the caller marks its list entry)
                constexpr bool kHandOn = !F32 && CF::VM > kVmax && CF::VM < kVmaxBig;
                const bool handed = kHandOn && (status & NS_CAPACITY);
                // sink mode: a node of the range left without a mesh
                if (SINK && !retry && !handed && n >= P.sink.n0 && n < P.sink.n1)
                    sink_add(P.sink, P.sink.node_part ? P.sink.node_part[n] : 0, 7, 1);
            }
            over_lanes<WL, CF::VM>(lane, 0, v - 1, [&](int l) { W.he_len[row + l] = 0; });
            return;
        }
        const int Msum = sh.wsum + NC, Fsum = sh.fsum;
        const int64_t rb = sh.rec;
        const int nent = sh.loop_base[v + 1];
        const int HX = NC + sh.wsum - V;
        const int64_t lw = SINK ? 0 : rec_loop_word(V, E, HX, rec_table_bytes(v, nent, WIDE));
        if constexpr (SINK) {
            over_lanes<WL, CF::VM>(lane, 0, v - 1, [&](int l) {
                W.he_len[row + l] = sh.loop_len[l + 1];
                W.he_loop[row + l] = rb >= 0 ? rb / 2 + sh.lbase[l + 1] : 0;
            });
            if (lane == 0) W.node_rec[n] = rb;
            if (n < P.sink.n0 || n >= P.sink.n1) return;  // halo node: its loops only
            sink_hash_node<T, CF>(P, sh, n, Msum, Fsum, pt_v, pt_x, pt_y, pt_z);
            return;
        }
        if (lane == 0) {
            W.node_cnt[NC_VERT * N + n] = V;
            W.node_cnt[NC_ARC * N + n] = E;
            W.node_cnt[NC_HOLE * N + n] = NC;
            W.node_cnt[NC_MESH * N + n] = Msum;
            W.node_cnt[NC_FAN * N + n] = Fsum;
            W.node_cnt[NC_STATUS * N + n] = 0;
            W.node_rec[n] = rb;
        }
        over_lanes<WL, CF::VM>(lane, 0, v - 1, [&](int l) {
            W.he_len[row + l] = sh.loop_len[l + 1];
            W.he_loop[row + l] = rb >= 0 ? (rb + lw) / 2 + sh.lbase[l + 1] : 0;
        });
        if (rb < 0) return;
        uint32_t *R = W.rec + rb;
        if (lane == 0) {
            R[0] = (uint32_t)V;
            R[1] = (uint32_t)E;
            R[2] = (uint32_t)NC;
            R[3] = (uint32_t)sh.ncirc;
            R[4] = (uint32_t)sh.wsum;
            R[5] = (uint32_t)Msum;
            R[6] = (uint32_t)Fsum;
            R[7] = (uint32_t)v | ((uint32_t)nent << 8) | (F32 ? 0u : kRecFp64) | (WIDE ? kRecWide : 0u);
        }
        // vertices and arcs as whole 16-byte groups (the record and both
        // blocks start on 16-byte boundaries)
        uint32_t *RV = R + kRecHead;
        for (int i = lane; i < V; i += WL)
            *(uint4 *)(RV + 4 * i) = make_uint4(sh.vname[i], __float_as_uint((float)sh.vx[i]),
                                                __float_as_uint((float)sh.vy[i]), __float_as_uint((float)sh.vz[i]));
        uint32_t *RA = RV + 4 * V;
        for (int j = lane; j < E; j += WL) {
            const ArcL<T> &A = sh.A[j];
            uint4 *dst = (uint4 *)(RA + kRecArcFields * j);
            auto fb = [](T x) { return __float_as_uint((float)x); };
            const uint32_t fwd = (A.full || A.ns <= A.ne) ? 1u : 0u;
            const uint32_t lower = sh.S[A.q].lower ? 1u : 0u;
            dst[0] = make_uint4(fb(A.o[0]), fb(A.o[1]), fb(A.o[2]), fb(A.a[0]));
            dst[1] = make_uint4(fb(A.a[1]), fb(A.a[2]), fb(A.b[0]), fb(A.b[1]));
            dst[2] = make_uint4(fb(A.b[2]), fb(A.t1), fb(A.dt),
                                (uint32_t)A.p | ((uint32_t)A.q << 8) | ((uint32_t)A.full << 16) | (fwd << 17) |
                                    (lower << 18));
            dst[3] = make_uint4((uint32_t)A.vs | ((uint32_t)A.ve << 16),
                                (uint32_t)A.nseg | (((uint32_t)A.contour & 0xffffu) << 16), (uint32_t)A.mbase,
                                (uint32_t)A.fbase);
        }
        uint32_t *RH = RA + kRecArcFields * E;
        for (int c = lane; c < NC; c += WL) {
            RH[3 * c] = __float_as_uint((float)sh.hc[c][0]);
            RH[3 * c + 1] = __float_as_uint((float)sh.hc[c][1]);
            RH[3 * c + 2] = __float_as_uint((float)sh.hc[c][2]);
        }
        // loop table (for re-subdivision at another resolution)
        using TabT = typename std::conditional<WIDE, uint16_t, uint8_t>::type;
        constexpr uint32_t kFwd = WIDE ? 0x8000u : 0x80u;
        TabT *RT = (TabT *)(R + rec_table_word(V, E, HX));
        over_lanes<WL, CF::VM>(lane, 0, v, [&](int l) { RT[l] = (TabT)sh.loop_base[l + 1]; });
        for (int e = lane; e < nent; e += WL) {
            const uint32_t ea = sh.entry_arc[e];
            RT[v + 1 + e] = (TabT)((ea & 0x7fffu) | ((ea & 0x8000u) ? kFwd : 0u));
        }
    }
}

template <typename T, typename CF, bool SINK = false>
__device__ __forceinline__ void node_body(const Params &P, Shared<T, CF> &sh, const int64_t n)
{
    constexpr int WL = CF::W;
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int NP = NPieces<T>::n;
    const T tp = Cst<T>::two_pi;
    const int lane = threadIdx.x & (WL - 1);
    const Work &W = P.w;
    const int64_t N = P.in.n_nodes;
    const int k = W.node_k ? (int)W.node_k[n] : P.k;
    const int64_t row = W.row[n];
    const int v = (int)(W.row[n + 1] - row);
    const float4 c4 = W.node4[n];
    const T rho = (T)c4.w;
    const V3<T> cen = v3((T)c4.x, (T)c4.y, (T)c4.z);
    if (lane == 0) {
        sh.status = 0;
        sh.n_arc = 0;
        sh.n_vert = 0;
        sh.n_contour = 0;
        sh.wsum = 0;
        sh.fsum = 0;
        sh.ncirc = 0;
        sh.rec = -1;
    }
    __syncthreads();
    if (v == 0 || v > CF::VM) {
        if (lane == 0) {
            for (int c = 0; c < kNodeCols; ++c) W.node_cnt[c * N + n] = 0;
            W.node_cnt[NC_STATUS * N + n] = v == 0 ? NS_ISOLATED : NS_VALENCE;
            W.node_rec[n] = -1;
            if (SINK && n >= P.sink.n0 && n < P.sink.n1)
                sink_add(P.sink, P.sink.node_part ? P.sink.node_part[n] : 0, 7, 1);
        }
        for (int i = lane; i < v; i += WL) W.he_len[row + i] = 0;
        return;
    }

    // ---- strut table -----------------------------------------------------
    over_lanes<WL, CF::VM>(lane, 0, v - 1, [&](int l) {
        int2 he = W.he[row + l];
        int far = he.x;
        float4 f4 = W.node4[far];
        bool bad;
        SL<T> s = strut_entry(cen, rho, v3((T)f4.x, (T)f4.y, (T)f4.z), (T)f4.w, (int)((int64_t)far > n), bad);
        s.sid = he.y;
        s.far = far;
        if (bad || far == n) atomicOr(&sh.status, NS_INVALID_STRUT);
        sh.S[l + 1] = s;
    });
    __syncthreads();
    over_lanes<WL, CF::VM>(lane, 0, v - 1, [&](int l) {
        for (int j = 0; j < v; ++j)
            if (j != l && sh.S[j + 1].far == sh.S[l + 1].far) atomicOr(&sh.status, NS_DUPLICATE);
    });
    if (F32 && lane == 0 && !(P.kappa_max > 0.f)) atomicOr(&sh.status, NS_PREC);  // all FP64
    __syncthreads();
    if (group_status<WL>(sh)) goto tail;

    // ---- conics, trimming, arcs and owned vertices ------------------------
    {
        const int nconic = v * (v + 1) / 2;
        for (int c0 = 0; c0 < nconic;) {
            // A last round of at most WL / 8 conics (v <= 8: at most 7
            // constraints each) runs on 8 lanes per conic, one constraint per
            // lane; the conic's first lane intersects the kept sets in
            // constraint order.  Otherwise one lane per conic.
            const bool split = F32 && WL >= 16 && v <= 8 && (nconic - c0) * 8 <= WL;
            const int ci = split ? c0 + (lane >> 3) : c0 + lane;
            const int sub = split ? (lane & 7) : 0;
            const bool grp = ci < nconic;
            const bool act = grp && sub == 0;
            c0 += split ? WL / 8 : WL;
            int p = 0, q = 0;
            if (grp) {
                int rem = ci;
                while (rem >= v - p) { rem -= v - p; ++p; }
                q = p + 1 + rem;
            }
            Con<T> C;
            TrimOut<T> TR;
            TR.n = 0;
            TR.full = 0;
            TR.ovf = 0;
            const bool ell = grp && conic_of(sh.S, rho, p, q, C);
            if (act && !ell) atomicOr(&sh.status, NS_NON_ELLIPTIC);
            // a conic far larger than the node (kept or not): its points and
            // the parameters of its ends would lose its size over rho in
            // relative FP32 precision, so the node goes to FP64 before any
            // of its conics is trimmed
            if (F32 && act && ell &&
                m_max(dot(C.o, C.o), dot(C.a, C.a)) > (T)(kConicMax * kConicMax) * rho * rho)
                atomicOr(&sh.status, NS_PREC);
            if (F32 && group_status<WL>(sh)) break;
            {
                const V3<T> gp = p ? gvec(sh.S[p]) : zero3<T>();
                const T hp = p ? sh.S[p].h : (T)0;
                // split: this lane's constraint, the sub-th label of 0..v
                // other than p and q (p < q)
                int myr = sub, mykind = 0;
                T mylo = (T)0, mylc = (T)0;
                if (split) {
                    if (myr >= p) ++myr;
                    if (myr >= q) ++myr;
                    if (ell && sub < v - 1) mykind = cons_interval(sh.S, gp, hp, myr, C, mylo, mylc);
                }
                const int nsteps = split ? 0 : (act && ell ? v + 1 : 0);
                TrimRun<T> st;
                if constexpr (F32) {
                    if (split) split_steps(st, mykind, myr, mylo, mylc, std::make_integer_sequence<int, 7>{});
                }
                for (int s2 = 0; s2 < nsteps; ++s2) {
                    int k2 = 0;
                    T lo2 = (T)0, lc2 = (T)0;
                    if (s2 != p && s2 != q) k2 = cons_interval(sh.S, gp, hp, s2, C, lo2, lc2);
                    trim_step(st, k2, lo2, lc2, s2);
                    if (st.done) break;
                }
                if (act && ell) {
                    trim_finish(sh.S, p, q, C, gp, hp, st, TR);
                    if (TR.ovf) atomicOr(&sh.status, F32 ? NS_PREC : NS_CAPACITY);
                }
            }
            // arcs of this conic, sorted by the smaller endpoint name
            uint32_t ns_[NP], ne_[NP], key[NP];
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                if (TR.full) {
                    ns_[i] = ne_[i] = vname3(p, q, 255, 0);
                } else {
                    ns_[i] = tie_name(p, q, TR.pc[i].rs, TR.pc[i].roots & 1);
                    ne_[i] = tie_name(p, q, TR.pc[i].re, (TR.pc[i].roots >> 1) & 1);
                }
                key[i] = i < TR.n ? (ns_[i] < ne_[i] ? ns_[i] : ne_[i]) : 0xffffffffu;
            }
            int ord[NP];
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                int rank = 0;
#pragma unroll
                for (int j = 0; j < NP; ++j) rank += (key[j] < key[i]) || (key[j] == key[i] && j < i);
                ord[i] = rank;
            }
            int cnt = act ? TR.n : 0, tot;
            int base = group_excl_scan<WL>(cnt, &tot) + sh.n_arc;
            if (sh.n_arc + tot > CF::AC) {
                if (lane == 0) atomicOr(&sh.status, NS_CAPACITY);
            } else {
#pragma unroll
                for (int i = 0; i < NP; ++i) {
                    if (i < cnt) {
                        ArcL<T> &A = sh.A[base + ord[i]];
                        A.o[0] = C.o.x; A.o[1] = C.o.y; A.o[2] = C.o.z;
                        A.a[0] = C.a.x; A.a[1] = C.a.y; A.a[2] = C.a.z;
                        A.b[0] = C.b.x; A.b[1] = C.b.y; A.b[2] = C.b.z;
                        A.p = p; A.q = q; A.full = TR.full;
                        if (TR.full) {
                            A.t1 = (T)0;
                            A.t2 = tp;
                            A.dt = tp;
                        } else {
                            piece_range(TR.pc[i], A.t1, A.t2, A.dt);
                        }
                        A.ns = ns_[i];
                        A.ne = ne_[i];
                    }
                }
            }
            // owned vertices: ties (p, q, r) with r > q, and whole-conic starts
            uint32_t on[2 * NP];
            T os_[2 * NP], oc_[2 * NP];
            int orr[2 * NP];
            int own = 0;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
#pragma unroll
                for (int end = 0; end < 2; ++end) {
                    bool mine = false;
                    uint32_t nm = 0;
                    T ds = (T)0, dc = (T)1;  // direction of the point: t = 0 for a whole conic
                    int r = -1;
                    if (i < cnt) {
                        if (TR.full) {
                            mine = (end == 0 && i == 0);
                            nm = ns_[i];
                        } else {
                            r = end ? TR.pc[i].re : TR.pc[i].rs;
                            mine = r > q;
                            nm = end ? ne_[i] : ns_[i];
                            ds = end ? TR.pc[i].es : TR.pc[i].ss;
                            dc = end ? TR.pc[i].ec : TR.pc[i].sc;
                        }
                    }
                    // drop repeats within the conic (degenerate tangencies)
#pragma unroll
                    for (int j = 0; j < 2 * NP; ++j)
                        if (j < own && on[j] == nm) mine = false;
#pragma unroll
                    for (int j = 0; j < 2 * NP; ++j)
                        if (mine && j == own) { on[j] = nm; os_[j] = ds; oc_[j] = dc; orr[j] = r; }
                    if (mine) ++own;
                }
            }
            int ntot;
            int vbase = group_excl_scan<WL>(own, &ntot) + sh.n_vert;
            if (sh.n_vert + ntot > CF::VC) {
                if (lane == 0) atomicOr(&sh.status, NS_CAPACITY);
            } else {
#pragma unroll
                for (int i = 0; i < 2 * NP; ++i) {
                    if (i < own) {
                        int rank = 0;
#pragma unroll
                        for (int j = 0; j < 2 * NP; ++j) rank += (j < own) && (on[j] < on[i]);
                        V3<T> w = conic_dir(C, os_[i], oc_[i]);
                        sh.vname[vbase + rank] = on[i];
                        sh.vx[vbase + rank] = w.x;
                        sh.vy[vbase + rank] = w.y;
                        sh.vz[vbase + rank] = w.z;
                        if (F32 && orr[i] >= 0 && !tie_trusted(sh.S, p, q, orr[i], w, rho, (T)P.kappa_max))
                            atomicOr(&sh.status, NS_PREC);
                    }
                }
            }
            __syncthreads();
            // advance the running counts (tot / ntot are wave-uniform)
            if (lane == 0) {
                if (sh.n_arc + tot <= CF::AC) sh.n_arc += tot;
                if (sh.n_vert + ntot <= CF::VC) sh.n_vert += ntot;
            }
            __syncthreads();
        }
    }
    if (group_status<WL>(sh)) goto tail;

    // ---- arc ends -> vertex indices, vertex degrees, segment counts -------
    {
        const int E = sh.n_arc, V = sh.n_vert;
        for (int j = lane; j < E; j += WL) {
            ArcL<T> &A = sh.A[j];
            A.vs = find_vert(sh, A.ns);
            A.ve = find_vert(sh, A.ne);
            if (A.vs < 0 || A.ve < 0) atomicOr(&sh.status, NS_TOPOLOGY);
            A.contour = -1;
        }
        // segment counts (Eq. 11)
        for (int i = lane; i < V; i += WL) sh.vdeg[i] = 0;
        __syncthreads();
        for (int j = lane; j < E; j += WL) {
            ArcL<T> &A = sh.A[j];
            if (A.full) {
                A.nseg = k;
            } else {
                T u = A.dt * ((T)k * Cst<T>::inv_two_pi);
                int ns = (int)m_floor(u) + 1;
                A.nseg = ns < k ? ns : k;
            }
        }
        for (int j = lane; j < E; j += WL) {
            const ArcL<T> &A = sh.A[j];
            if (A.full || A.vs < 0 || A.ve < 0) continue;
            atomicAdd(&sh.vdeg[A.vs], 1);
            atomicAdd(&sh.vdeg[A.ve], 1);
        }
        __syncthreads();
        for (int i = lane; i < V; i += WL)
            if ((sh.vname[i] & 0xff00u) != 0xff00u && sh.vdeg[i] != 3) atomicOr(&sh.status, NS_TOPOLOGY);
        __syncthreads();
        if (group_status<WL>(sh)) goto tail;
    }

    // ---- end loops per strut ----------------------------------------------
    // Every arc lies on the loops of its two labels p, q (one loop for a
    // tangency circle).  Lanes over (arc, side) memberships: orientation
    // along the strut angle, successor by shared vertex, then the position
    // in the loop counted from the arc whose loop-start vertex has the
    // smallest name.
    {
        const int E = sh.n_arc;
        over_lanes<WL, CF::VM>(lane, 0, v, [&](int l) {
            sh.loop_cnt[l] = 0;
            sh.loop_len[l] = 0;
            sh.loop_full[l] = 0;
        });
        __syncthreads();
        for (int j = lane; j < E; j += WL) {
            const ArcL<T> &A = sh.A[j];
            if (A.p) atomicAdd(&sh.loop_cnt[A.p], 1);
            atomicAdd(&sh.loop_cnt[A.q], 1);
        }
        __syncthreads();
        if constexpr (WL > CF::VM + 1) {
            int c = (lane >= 1 && lane <= v) ? sh.loop_cnt[lane] : 0, tot;
            int base = group_excl_scan<WL>(c, &tot);
            if (lane >= 1 && lane <= v) sh.loop_base[lane] = base;
            if (lane == 0) sh.loop_base[v + 1] = tot;
        } else if (lane == 0) {
            int acc = 0;
            for (int m = 1; m <= v; ++m) {
                sh.loop_base[m] = acc;
                acc += sh.loop_cnt[m];
            }
            sh.loop_base[v + 1] = acc;
        }
        __syncthreads();
        over_lanes<WL, CF::VM>(lane, 0, v, [&](int l) { sh.loop_cnt[l] = 0; });  // reused as fill cursor
        __syncthreads();
        for (int j = lane; j < E; j += WL) {
            const ArcL<T> &A = sh.A[j];
            T tm = A.t1 + (T)0.5 * A.dt;
            T st, ct;
            m_sincos(tm, &st, &ct);
            Con<T> C = arc_con(A);
            V3<T> w = C.o + C.a * st + C.b * ct;
            V3<T> dw = C.a * ct - C.b * st;
            V3<T> wdw = cross(w, dw);
            for (int side = 0; side < 2; ++side) {
                int m = side ? A.q : A.p;
                if (m == 0) continue;
                const SL<T> &s = sh.S[m];
                int pp = sh.loop_base[m] + atomicAdd(&sh.loop_cnt[m], 1);
                const int dir = dot(wdw, v3(s.sx, s.sy, s.sz)) > (T)0 ? 1 : -1;
                sh.loop_arc[pp] = (uint8_t)j;
                sh.loop_dir[pp] = (int8_t)dir;
                // start name and loop of the membership, kept in entry_off /
                // entry_m (free until the tail lays out the loop samples)
                sh.entry_off[pp] = (int)(dir > 0 ? A.ns : A.ne);
                sh.entry_m[pp] = (uint8_t)m;
                atomicAdd(&sh.loop_len[m], A.nseg);
                if (A.full) atomicAdd(&sh.loop_full[m], 1);
            }
        }
        __syncthreads();
        const int tot = sh.loop_base[v + 1];
        auto sname = [&](int pp) { return (uint32_t)sh.entry_off[pp]; };
        auto ename = [&](int pp) {
            const ArcL<T> &A = sh.A[sh.loop_arc[pp]];
            return sh.loop_dir[pp] > 0 ? A.ne : A.ns;
        };
        auto strut_of = [&](int pp) { return (int)sh.entry_m[pp]; };
        for (int pp = lane; pp < tot; pp += WL) {
            const int m = strut_of(pp);
            const int b0 = sh.loop_base[m], b1 = sh.loop_base[m + 1];
            const uint32_t en = ename(pp), sn = sname(pp);
            int nxt = -1, hits = 0;
            bool first = true;
            for (int q2 = b0; q2 < b1; ++q2) {
                uint32_t s2 = sname(q2);
                if (s2 == en) { nxt = q2; ++hits; }
                if (s2 < sn || (s2 == sn && q2 < pp)) first = false;
            }
            if (hits != 1) atomicOr(&sh.status, NS_LOOP);
            sh.loop_next[pp] = (uint16_t)(nxt < 0 ? pp : nxt);
            if (first) sh.loop_first[m] = pp;
        }
        over_lanes<WL, CF::VM>(lane, 1, v, [&](int l) {
            const int c = sh.loop_base[l + 1] - sh.loop_base[l];
            if (c == 0 || (sh.loop_full[l] && c != 1)) atomicOr(&sh.status, NS_LOOP);
        });
        __syncthreads();
        if (group_status<WL>(sh)) goto tail;
        // position of each arc in its loop.  Every arc reached within c - 1
        // steps from the first makes the chain a path through all c arcs; it
        // closes into one loop exactly when the arc reached last leads back
        // to the first.
        for (int pp = lane; pp < tot; pp += WL) {
            const int m = strut_of(pp);
            const int b0 = sh.loop_base[m], c = sh.loop_base[m + 1] - b0;
            int cur = sh.loop_first[m], t = 0;
            while (cur != pp && t < c) {
                cur = sh.loop_next[cur];
                ++t;
            }
            if (t >= c) {
                atomicOr(&sh.status, NS_LOOP);
                continue;
            }
            sh.loop_ord[b0 + t] = (uint8_t)(pp - b0);
            if (t == c - 1 && sh.loop_next[pp] != sh.loop_first[m]) atomicOr(&sh.status, NS_LOOP);
        }
        if (tot > 2 * CF::AC && lane == 0) atomicOr(&sh.status, NS_CAPACITY);
        __syncthreads();
        if (group_status<WL>(sh)) goto tail;
    }

    // ---- hole contours ------------------------------------------------------
    {
        const int E = sh.n_arc;
        int ncirc = 0;
        while (ncirc < E && sh.A[ncirc].p == 0) ++ncirc;  // circular arcs sort first
        for (int i = lane; i < ncirc; i += WL) {
            const ArcL<T> &A = sh.A[i];
            uint32_t lab = A.ns < A.ne ? A.ns : A.ne;
            if (!A.full) {
                int cur = i, from = A.vs, steps = 0;
                while (true) {
                    const ArcL<T> &B = sh.A[cur];
                    int to = B.vs == from ? B.ve : B.vs;
                    uint32_t tn = sh.vname[to];
                    if (tn < lab) lab = tn;
                    int nxt = -1, hits = 0;
                    for (int j = 0; j < ncirc; ++j) {
                        if (j == cur || sh.A[j].full) continue;
                        if (sh.A[j].vs == to || sh.A[j].ve == to) { nxt = j; ++hits; }
                    }
                    if (hits != 1 || ++steps > ncirc) { atomicOr(&sh.status, NS_TOPOLOGY); break; }
                    from = to;
                    cur = nxt;
                    if (cur == i) break;
                }
            }
            sh.clabel[i] = lab;
        }
        __syncthreads();
        for (int i = lane; i < ncirc; i += WL) {
            uint32_t lab = sh.clabel[i];
            int rank = 0;
            for (int j = 0; j < ncirc; ++j) {
                uint32_t lj = sh.clabel[j];
                bool first = true;
                for (int t = 0; t < j; ++t)
                    if (sh.clabel[t] == lj) first = false;
                if (first && lj < lab) ++rank;
            }
            sh.A[i].contour = rank;
            bool first = true;
            for (int t = 0; t < i; ++t)
                if (sh.clabel[t] == lab) first = false;
            if (first) atomicAdd(&sh.n_contour, 1);
        }
        __syncthreads();
        if (lane == 0 && sh.n_vert - sh.n_arc + sh.n_contour != 2 - v) atomicOr(&sh.status, NS_TOPOLOGY);
        __syncthreads();
        if (group_status<WL>(sh)) goto tail;
    }

tail:
    node_tail<T, CF, SINK>(P, sh, n, k, v, row, rho, cen);
}

// Re-subdivision at resolution k of a node whose meta-mesh is in a record
// written at another resolution (the paper's reusable meta-mesh, Alg. 1):
// arcs, vertices, end-loop order and hole contours are read back; segment
// counts (Eq. 11), points (Eq. 12), hole centres (Eq. 13) and end-loop
// samples are redone by the tail.  Only FP32 meta-meshes are reused: a node
// the FP32 path did not settle at the source resolution (meshed in FP64, or
// not meshed) goes to the class's redo list and is solved again from the
// lattice, so that every node takes the path, and gives the result, of a
// forward pass at k.  All record words are loaded in one round (one arc,
// one vertex and one table word per lane: E <= AC = W, V <= VC <= W) before
// anything is written to LDS.
template <typename CF>
__device__ __forceinline__ void node_retri(const Params &P, Shared<float, CF> &sh, const int64_t n, const int cls)
{
    using T = float;
    constexpr int WL = CF::W;
    static_assert(CF::AC == WL && CF::VC <= WL && (1 + CF::VM + 2 * CF::AC + 3) / 4 <= 2 * CF::AC + 1,
                  "one arc, vertex and table word per lane; the table is staged in entry_off");
    const int lane = threadIdx.x & (WL - 1);
    const Work &W = P.w;
    const int k = W.node_k ? (int)W.node_k[n] : P.k;
    const int64_t row = W.row[n];
    const int v = (int)(W.row[n + 1] - row);
    const float4 c4 = W.node4[n];
    const int64_t sb = P.src_node_rec[n];
    int2 he = make_int2(0, 0);
    if (lane < v) he = W.he[row + lane];
    const uint32_t *R = sb >= 0 ? P.src_rec + sb : nullptr;
    uint32_t h0 = 0, h1 = 0, h2 = 0, h4 = 0, h7 = 0;
    if (R) {
        h0 = R[0];
        h1 = R[1];
        h2 = R[2];
        h4 = R[4];  // first hole-centre index: V + interior points
        h7 = R[7];
    }
    const int V = (int)h0, E = (int)h1, NC = (int)h2, nent = (int)((h7 >> 8) & 0xffffu);
    if (!R || (h7 >> 24) || v == 0 || v > CF::VM || E > CF::AC || V > CF::VC || nent > 2 * CF::AC ||
        NC > CF::AC) {
        if (lane == 0) P.redo[W.cls_info[4 + cls] + atomicAdd(&P.redo_cnt[cls], 1)] = (int32_t)n;
        return;
    }
    // the record: vertices, arcs, loop table (all independent loads)
    const uint32_t *RV = R + kRecHead;
    const uint32_t *RA = RV + 4 * V;
    const uint32_t *RT = R + rec_table_word(V, E, NC + (int)h4 - V);
    const int twords = (v + 1 + nent + 3) >> 2;
    float4 f4 = c4;
    if (lane < v) f4 = W.node4[he.x];
    uint4 vq = make_uint4(0, 0, 0, 0);
    if (lane < V) vq = *(const uint4 *)(RV + 4 * lane);
    const uint32_t vw[4] = {vq.x, vq.y, vq.z, vq.w};
    uint4 aq[4] = {};
    if (lane < E)
        for (int f = 0; f < 4; ++f) aq[f] = ((const uint4 *)(RA + kRecArcFields * lane))[f];
    const uint32_t aw[14] = {aq[0].x, aq[0].y, aq[0].z, aq[0].w, aq[1].x, aq[1].y, aq[1].z,
                             aq[1].w, aq[2].x, aq[2].y, aq[2].z, aq[2].w, aq[3].x, aq[3].y};
    const uint32_t tw = lane < twords ? RT[lane] : 0u;

    const T rho = (T)c4.w;
    const V3<T> cen = v3((T)c4.x, (T)c4.y, (T)c4.z);
    if (lane < v) {
        bool bad;
        SL<T> st = strut_entry(cen, rho, v3((T)f4.x, (T)f4.y, (T)f4.z), (T)f4.w, (int)((int64_t)he.x > n), bad);
        st.sid = he.y;
        st.far = he.x;
        sh.S[lane + 1] = st;
    }
    if (lane < V) {
        sh.vname[lane] = vw[0];
        sh.vx[lane] = __uint_as_float(vw[1]);
        sh.vy[lane] = __uint_as_float(vw[2]);
        sh.vz[lane] = __uint_as_float(vw[3]);
    }
    if (lane < twords) sh.entry_off[lane] = (int)tw;  // staging; the tail rewrites entry_off
    if (lane == 0) {
        sh.status = 0;
        sh.wsum = 0;
        sh.fsum = 0;
        sh.ncirc = 0;
        sh.rec = -1;
        sh.loop_base[0] = 0;
        sh.n_arc = E;
        sh.n_vert = V;
        sh.n_contour = NC;
    }
    __syncthreads();
    if (lane < E) {
        ArcL<T> &A = sh.A[lane];
        for (int d = 0; d < 3; ++d) {
            A.o[d] = __uint_as_float(aw[d]);
            A.a[d] = __uint_as_float(aw[3 + d]);
            A.b[d] = __uint_as_float(aw[6 + d]);
        }
        A.t1 = __uint_as_float(aw[9]);
        A.dt = __uint_as_float(aw[10]);
        A.t2 = A.t1 + A.dt;
        const uint32_t u0 = aw[11], u1 = aw[12], u2 = aw[13];
        A.p = (int)(u0 & 0xffu);
        A.q = (int)((u0 >> 8) & 0xffu);
        A.full = (int)((u0 >> 16) & 1u);
        A.vs = (int)(u1 & 0xffffu);
        A.ve = (int)(u1 >> 16);
        A.ns = sh.vname[A.vs];
        A.ne = sh.vname[A.ve];
        A.contour = (u2 >> 16) == 0xffffu ? -1 : (int)(u2 >> 16);
        // Eq. 11 at the new resolution
        if (A.full) {
            A.nseg = k;
        } else {
            T u = A.dt * ((T)k * Cst<T>::inv_two_pi);
            int ns = (int)m_floor(u) + 1;
            A.nseg = ns < k ? ns : k;
        }
    }
    // loop table bytes: loop start of labels 1..v+1, then the entries
    auto tbyte = [&](int i) -> int { return (int)(((uint32_t)sh.entry_off[i >> 2] >> (8 * (i & 3))) & 0xffu); };
    if (lane <= v) sh.loop_base[lane + 1] = tbyte(lane);
    // entries in loop order: entry e is the (e - start)-th arc of its loop
    for (int e = lane; e < nent; e += WL) {
        const int b = tbyte(v + 1 + e);
        int m = 1;
        while (tbyte(m) <= e) ++m;  // loop_base[m + 1] = tbyte(m)
        sh.loop_arc[e] = (uint8_t)(b & 0x7f);
        sh.loop_dir[e] = (b & 0x80) ? 1 : -1;
        sh.loop_ord[e] = (uint8_t)(e - tbyte(m - 1));  // loop_base[m] = tbyte(m - 1)
    }
    __syncthreads();
    if (lane >= 1 && lane <= v) {
        int len = 0;
        for (int e = sh.loop_base[lane]; e < sh.loop_base[lane + 1]; ++e) len += sh.A[sh.loop_arc[e]].nseg;
        sh.loop_len[lane] = len;
    }
    __syncthreads();
    node_tail<T, CF, false>(P, sh, n, k, v, row, rho, cen);
}

// FP32, one valence class: a persistent loop takes items of 64 / W queued
// nodes from the class's work counter; every wave leaves once the counter has
// passed the class's last item.  MODE 0: meta-meshing of the queue; 1:
// re-subdivision of the queue; 2: meta-meshing of the redo list that mode 1
// left (its length is read on the device); 3: meta-meshing of the queue in
// sink mode (end loops kept, vertices and fans hashed).
enum { kModeMesh = 0, kModeRetri = 1, kModeRedo = 2, kModeSink = 3 };

// Guided self-scheduling on a work counter shared by the grid: a block takes
// a share of the items left (half of them over the grid, from what its last
// grab saw), at least one and at most kGrabMax, as the range [first, end).  The counter is one address for the whole chip and its
// atomics are serialised there: one per item throttled the node pass (a
// pass without the trimming, the re-subdivision, took as long as a full
// one); a few per block do not, and the last grabs are still single items.
// Block-uniform; every thread of the block calls it.  Blocks at or beyond
// the item count take nothing (a short list leaves most of the grid idle
// without an atomic each).
constexpr int kGrabMax = 16;
__device__ inline bool grab_items(int32_t *ctr, int64_t items, int64_t &seen, int *s_grab, int64_t &first,
                                  int64_t &end)
{
    if ((int64_t)blockIdx.x >= items) return false;
    if (threadIdx.x == 0) {
        int64_t g = (items - seen) / (2 * (int64_t)gridDim.x);
        g = g < 1 ? 1 : (g > kGrabMax ? kGrabMax : g);
        s_grab[0] = atomicAdd(ctr, (int)g);
        s_grab[1] = (int)g;
    }
    __syncthreads();
    first = s_grab[0];
    const int g = s_grab[1];
    __syncthreads();
    seen = first + g;
    end = seen < items ? seen : items;
    return first < items;
}

template <typename C, int MODE>
__device__ inline void drain_class(const Params &P, int cls, Shared<float, C> *sh, int *s_grab)
{
    constexpr int NPW = 64 / C::W;
    const int slot = threadIdx.x / C::W;
    const int64_t cnt = MODE == kModeRedo ? (int64_t)P.redo_cnt[cls] : P.w.cls_info[cls];
    const int64_t base = P.w.cls_info[4 + cls];
    const int32_t *list = MODE == kModeRedo ? P.redo : P.w.queue;
    int32_t *ctr = MODE == kModeRedo ? P.redo_ctr : P.w.work_ctr;
    const int64_t items = (cnt + NPW - 1) / NPW;
    int64_t seen = 0, first, end;
    while (grab_items(&ctr[cls], items, seen, s_grab, first, end)) {
        for (int64_t item = first; item < end; ++item) {
            const int64_t qi = item * NPW + slot;
            if (qi < cnt) {
                const int64_t node = list[base + qi];
                if (MODE == kModeRetri) node_retri<C>(P, sh[slot], node, cls);
                else if (MODE == kModeSink) node_body<float, C, true>(P, sh[slot], node);
                else node_body<float, C>(P, sh[slot], node);
            }
            __syncthreads();
        }
    }
}

// At most 168 VGPRs: three waves per SIMD (LDS allows as many), where one
// register more would leave two.
template <typename C, int MODE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) k_node32(Params P, int cls)
{
    __shared__ Shared<float, C> sh[64 / C::W];
    __shared__ int s_grab[2];
    drain_class<C, MODE>(P, cls, sh, s_grab);
}

// The classes v <= 4 (four nodes per wave) and 5..8 (two) in one persistent
// launch, the heavier first: the light nodes fill the tail of the others
// instead of running as a short launch of their own.  The two LDS layouts
// share one block of LDS, used by one class at a time.
union SharedV4V8 {
    Shared<float, CfgV8> b[2];
    Shared<float, CfgV4> a[4];
};
template <int MODE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) k_node32_v8v4(Params P)
{
    __shared__ SharedV4V8 sh;
    __shared__ int s_grab[2];
    drain_class<CfgV8, MODE>(P, 1, sh.b, s_grab);
    drain_class<CfgV4, MODE>(P, 0, sh.a, s_grab);
}

// The multi-wave class: one node per block of kBigWaves waves, items from the
// class's work counter as above.  Re-subdivision does not read these nodes'
// records: they are queued for a full solve (MODE 1), which MODE 2 runs.
template <int MODE>
__global__ void __launch_bounds__(64 * kBigWaves) k_node32_big(Params P)
{
    constexpr int cls = 3;
    __shared__ Shared<float, CfgBig> sh;
    __shared__ int s_grab[2];
    const int64_t cnt = MODE == kModeRedo ? (int64_t)P.redo_cnt[cls] : P.w.cls_info[cls];
    const int64_t base = P.w.cls_info[4 + cls];
    const int32_t *list = MODE == kModeRedo ? P.redo : P.w.queue;
    int32_t *ctr = MODE == kModeRedo ? P.redo_ctr : P.w.work_ctr;
    int64_t seen = 0, first, end;
    while (grab_items(&ctr[cls], cnt, seen, s_grab, first, end)) {
        for (int64_t item = first; item < end; ++item) {
            const int64_t node = list[base + item];
            if (MODE == kModeRetri) {
                if (threadIdx.x == 0) P.redo[base + atomicAdd(&P.redo_cnt[cls], 1)] = (int32_t)node;
            } else if (MODE == kModeSink) {
                node_body<float, CfgBig, true>(P, sh, node);
            } else {
                node_body<float, CfgBig>(P, sh, node);
            }
            __syncthreads();
        }
    }
}

// Thread-centric ablation: every lane meshes a node of its own (64 nodes per
// wave in node id order, no valence classes, the full capacities), with the
// per-node scratch that the kernel above keeps in LDS in global memory —
// the design the paper compares its warp-centric one against.  Same code,
// one lane per node: the results are those of the wave-centric pass.
using CfgT1 = Cfg<kVmaxBig, kAcapBig, kVcapBig, 1>;
__global__ void __launch_bounds__(64) k_node32_thread(Params P, Shared<float, CfgT1> *scratch)
{
    const int64_t N = P.in.n_nodes;
    Shared<float, CfgT1> &sh = scratch[(int64_t)blockIdx.x * 64 + threadIdx.x];
    for (int64_t n = (int64_t)blockIdx.x * 64 + threadIdx.x; n < N; n += (int64_t)gridDim.x * 64)
        node_body<float, CfgT1>(P, sh, n);
}

// FP64: the nodes the FP32 pass handed over, looped over by a fixed grid
// (also after a re-subdivision: these nodes are solved in full).  One
// instantiation takes the nodes of up to kVmax struts (a wave per node), the
// other the multi-wave class (a block of kBigWaves waves per node).
// At most 256 registers (VGPRs and AGPRs together): two waves per SIMD.
template <typename C, bool SINK>
__global__ void __launch_bounds__(C::W) __attribute__((amdgpu_waves_per_eu(2))) k_node64(Params P)
{
    __shared__ Shared<double, C> sh;
    __shared__ int s_grab[2];
    // the kernel's class: 0 one wave (v <= kVmax), 1 two waves (v <= kVmaxMid),
    // 2 four waves; the launches run in that order
    constexpr int cls = C::VM <= kVmax ? 0 : (C::VM <= kVmaxMid ? 1 : 2);
    constexpr int ctr = cls == 0 ? 4 : (cls == 1 ? 6 : 5);
    const int64_t cnt = P.w.flags[2];
    // guided grabs over the hand-over list (its nodes differ in cost)
    int64_t seen = 0, first, end;
    while (grab_items(&P.w.work_ctr[ctr], cnt, seen, s_grab, first, end)) {
        for (int64_t i = first; i < end; ++i) {
            // an entry the two-wave kernel could not hold is stored negated
            // (~node): the four-wave kernel takes it whatever its valence
            const int32_t e = P.w.fb_list[i];
            const int64_t node = e < 0 ? ~e : e;
            const int64_t v = P.w.row[node + 1] - P.w.row[node];
            const int ncls = e < 0 ? 2 : (v <= kVmax ? 0 : (v <= kVmaxMid ? 1 : 2));
            if (ncls == cls) {
                node_body<double, C, SINK>(P, sh, node);
                if constexpr (cls == 1) {
                    __syncthreads();
                    if (threadIdx.x == 0 && (sh.status & NS_CAPACITY)) P.w.fb_list[i] = ~(int32_t)node;
                }
            }
            __syncthreads();
        }
    }
}

constexpr unsigned kFp64Grid = 2048;
constexpr unsigned kFp64MidGrid = 1024;
constexpr unsigned kFp64BigGrid = 512;
constexpr int64_t kBigGrid = 2048;  // blocks of a multi-wave class launch
// waves of a one-wave-class launch: as many as the chip holds at once (256
// compute units, 12 blocks of 64 threads each by LDS)
constexpr int64_t kNodeGrid = 256 * 12;
constexpr int64_t kRedoGrid = 512;       // waves of that launch over a redo list
constexpr int64_t kMinGrid = 32;         // blocks of a class launch sized by an estimate

}  // namespace

constexpr int64_t kThreadGrid = 2048;  // blocks of the thread-centric pass

size_t node_thread_scratch_bytes() { return sizeof(Shared<float, CfgT1>) * (size_t)kThreadGrid * 64; }

hipError_t launch_node_thread(const Inputs &in, const Work &w, int k, float kappa_max, void *scratch,
                              hipStream_t st)
{
    if (in.n_nodes == 0) return hipSuccess;
    Params P;
    P.in = in;
    P.w = w;
    P.k = k;
    P.kappa_max = kappa_max;
    P.src_rec = nullptr;
    P.src_node_rec = nullptr;
    P.redo = nullptr;
    P.redo_cnt = nullptr;
    P.redo_ctr = nullptr;
    P.sink = SinkOut{};
    const int64_t blocks = (in.n_nodes + 63) / 64;
    k_node32_thread<<<(unsigned)(blocks < kThreadGrid ? blocks : kThreadGrid), 64, 0, st>>>(
        P, (Shared<float, CfgT1> *)scratch);
    return hipGetLastError();
}

hipError_t launch_node(const Inputs &in, const Work &w, int k, float kappa_max, int fp64, hipStream_t st,
                       const uint32_t *src_rec, const int64_t *src_node_rec, int32_t *redo, int32_t *redo_cnt,
                       const SinkOut *sink, const int64_t *cls_est)
{
    if (in.n_nodes == 0) return hipSuccess;
    Params P;
    P.sink = sink ? *sink : SinkOut{};
    P.in = in;
    P.w = w;
    P.k = k;
    P.kappa_max = kappa_max;
    P.src_rec = src_rec;
    P.src_node_rec = src_node_rec;
    P.redo = redo;
    P.redo_cnt = redo_cnt;
    P.redo_ctr = redo_cnt ? redo_cnt + 4 : nullptr;
    if (fp64) {
        if (sink) {
            k_node64<CfgV16, true><<<kFp64Grid, 64, 0, st>>>(P);
            k_node64<CfgMid, true><<<kFp64MidGrid, CfgMid::W, 0, st>>>(P);
            k_node64<CfgBig, true><<<kFp64BigGrid, CfgBig::W, 0, st>>>(P);
        } else {
            k_node64<CfgV16, false><<<kFp64Grid, 64, 0, st>>>(P);
            k_node64<CfgMid, false><<<kFp64MidGrid, CfgMid::W, 0, st>>>(P);
            k_node64<CfgBig, false><<<kFp64BigGrid, CfgBig::W, 0, st>>>(P);
        }
        return hipGetLastError();
    }
    // persistent grids: enough waves to fill the chip, never more than
    // items; with a class estimate, sized by the class (at least a few
    // blocks, so that an estimate grown stale still drains the queue)
    auto items_of = [&](int cls, int npw) {
        const int64_t nodes = cls_est ? cls_est[cls] : in.n_nodes;
        return (nodes + npw - 1) / npw;
    };
    auto clampg = [&](int64_t items, int64_t cap) {
        const int64_t lo = cls_est ? kMinGrid : 1;
        items = items < lo ? lo : items;
        return (unsigned)(items < cap ? items : cap);
    };
    // classes 0 and 1 share a launch: items of both
    const int64_t light = items_of(0, 4) + items_of(1, 2);
    const unsigned g01 = clampg(light, kNodeGrid), g01_redo = clampg(light, kRedoGrid);
    const unsigned g2 = clampg(items_of(2, 1), kNodeGrid), g2_redo = clampg(items_of(2, 1), kRedoGrid);
    const unsigned big_grid = clampg(items_of(3, 1), kBigGrid);
    if (src_rec) {
        if (!redo || !redo_cnt) return hipErrorInvalidValue;
        k_node32_v8v4<kModeRetri><<<g01, 64, 0, st>>>(P);
        k_node32<CfgV16, kModeRetri><<<g2, 64, 0, st>>>(P, 2);
        k_node32_big<kModeRetri><<<big_grid, CfgBig::W, 0, st>>>(P);
        // the redo lists are short unless most nodes needed FP64 at the source
        k_node32_v8v4<kModeRedo><<<g01_redo, 64, 0, st>>>(P);
        k_node32<CfgV16, kModeRedo><<<g2_redo, 64, 0, st>>>(P, 2);
        k_node32_big<kModeRedo><<<big_grid, CfgBig::W, 0, st>>>(P);
    } else if (sink) {
        k_node32_v8v4<kModeSink><<<g01, 64, 0, st>>>(P);
        k_node32<CfgV16, kModeSink><<<g2, 64, 0, st>>>(P, 2);
        k_node32_big<kModeSink><<<big_grid, CfgBig::W, 0, st>>>(P);
    } else {
        k_node32_v8v4<kModeMesh><<<g01, 64, 0, st>>>(P);
        k_node32<CfgV16, kModeMesh><<<g2, 64, 0, st>>>(P, 2);
        k_node32_big<kModeMesh><<<big_grid, CfgBig::W, 0, st>>>(P);
    }
    return hipGetLastError();
}

}  // namespace lm
