// Lossy 128-bit arc codec (the compressive arc representation of Sec.
// 4.2.1, error bound Eq. 5).  An arc x(t) = c + a sin t + b cos t,
// t in [t1, t2] (node-local) keeps: a as (r, theta, phi) on 12 / 15 / 16
// bits with r in [R_min, 4 R_max]; the length of b on 12 bits in
// [0.1 R_min, R_max] (its direction is a x d / |a x d| for a reference
// direction d recomputed from the lattice: the strut's own direction for a
// tangency circle, the normal (g_p - g_q) / |g_p - g_q| of the seam plane
// for an ellipse); c as (r, theta, phi) with r in [0, R_max]; t1 on 15 bits
// over [0, 2 pi) and the span t2 - t1 on 15 bits over [0, 2 pi].  Fields go
// least significant bit first into four 32-bit words in that order.  An arc
// outside these ranges, or whose b does not lie where a x d puts it, is kept
// whole in a fallback list (its code then holds the list slot).
//
// Quantisation decides integers, so the encoder computes in FP64 and this
// file is compiled without floating-point contraction.
#include <math.h>

#include "common.h"

namespace lm {
namespace {

constexpr int kNr = 12, kMth = 15, kMph = 16, kNt = 15;
constexpr double kPi = 3.14159265358979323846;

struct D3 {
    double x, y, z;
};
__device__ inline D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__device__ inline D3 sub(D3 a, D3 b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline D3 scl(D3 a, double s) { return d3(a.x * s, a.y * s, a.z * s); }
__device__ inline D3 dvd(D3 a, double s) { return d3(a.x / s, a.y / s, a.z / s); }
__device__ inline double nrm(D3 a) { return sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }
__device__ inline D3 crs(D3 a, D3 b)
{
    return d3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

struct CodecArgs {
    Inputs in;
    Work w;
    const float *arc;       // [11][ld]
    const uint32_t *u32;    // [3][ld]: p | q << 8 | whole << 16, ends, node
    int64_t E, ld;
    double rmin, rmax;
    uint32_t *codes;        // [E][4]
    uint32_t *mask;         // [(E + 31) / 32]
    float *fb;              // [fb_cap][11]
    int64_t fb_cap;
    unsigned long long *fb_n;
    float *out;             // decode: [11][ld_out]
    int64_t ld_out;
};

// strut of label lab (1..v) at node n: g = e / kappa and the canonical
// direction (lower -> higher node id), in FP64
__device__ inline void strut_g(const CodecArgs &A, int64_t n, int lab, D3 &g, D3 &es)
{
    const int2 he = A.w.he[A.w.row[n] + lab - 1];
    const float4 c = A.w.node4[n], f = A.w.node4[he.x];
    const D3 xn = d3(c.x, c.y, c.z), xf = d3(f.x, f.y, f.z);
    const D3 dv = sub(xf, xn);
    const double L = nrm(dv);
    const D3 e = dvd(dv, L);
    const double sig = ((double)c.w - (double)f.w) / L;
    const double kap = sqrt((1.0 - sig) * (1.0 + sig));
    g = dvd(e, kap);
    const bool lower = (int64_t)he.x > n;
    const D3 d = lower ? sub(xf, xn) : sub(xn, xf);
    es = dvd(d, nrm(d));
}

__device__ inline D3 ref_dir(const CodecArgs &A, int64_t j)
{
    const uint32_t u0 = A.u32[j];
    const int p = (int)(u0 & 0xffu), q = (int)((u0 >> 8) & 0xffu);
    const int64_t n = (int64_t)A.u32[2 * A.ld + j];
    D3 gq, esq;
    strut_g(A, n, q, gq, esq);
    if (p == 0) return esq;
    D3 gp, esp;
    strut_g(A, n, p, gp, esp);
    const D3 nv = sub(gp, gq);
    return dvd(nv, nrm(nv));
}

__device__ inline uint32_t qlin(double v, double lo, double hi, int bits)
{
    const double levels = (double)((1 << bits) - 1);
    double s = (v - lo) / (hi - lo) * levels;
    s = s < 0.0 ? 0.0 : (s > levels ? levels : s);
    return (uint32_t)rint(s);
}
__device__ inline double dlin(uint32_t q, double lo, double hi, int bits)
{
    return lo + (double)q * (hi - lo) / (double)((1 << bits) - 1);
}
__device__ inline uint32_t qper(double ang, int bits)
{
    const double n = (double)(1u << bits);
    return (uint32_t)(int64_t)rint(ang / (2.0 * kPi) * n) & ((1u << bits) - 1);
}
__device__ inline double dper(uint32_t q, int bits) { return (double)q * (2.0 * kPi) / (double)(1u << bits); }

__device__ inline void sph(D3 v, double &r, double &th, double &ph)
{
    r = nrm(v);
    double z = r > 0.0 ? v.z / r : 1.0;
    z = z < -1.0 ? -1.0 : (z > 1.0 ? 1.0 : z);
    th = acos(z);
    ph = atan2(v.y, v.x);
    if (ph < 0.0) ph = ph + 2.0 * kPi;
}
__device__ inline D3 cart(double r, double th, double ph)
{
    return scl(d3(sin(th) * cos(ph), sin(th) * sin(ph), cos(th)), r);
}

struct Bits {
    unsigned long long lo = 0, hi = 0;
    int pos = 0;
    __device__ void put(uint32_t v, int bits)
    {
        const unsigned long long x = (unsigned long long)v;
        if (pos >= 64) {
            hi |= x << (pos - 64);
        } else {
            lo |= x << pos;
            if (pos + bits > 64) hi |= x >> (64 - pos);
        }
        pos += bits;
    }
    __device__ uint32_t get(int bits)
    {
        unsigned long long x;
        if (pos >= 64) {
            x = hi >> (pos - 64);
        } else {
            x = lo >> pos;
            if (pos + bits > 64) x |= hi << (64 - pos);
        }
        pos += bits;
        return (uint32_t)(x & ((1ull << bits) - 1));
    }
};

__global__ void k_arc_encode(CodecArgs A)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= A.E) return;
    const D3 c = d3(A.arc[j], A.arc[A.ld + j], A.arc[2 * A.ld + j]);
    const D3 a = d3(A.arc[3 * A.ld + j], A.arc[4 * A.ld + j], A.arc[5 * A.ld + j]);
    const D3 b = d3(A.arc[6 * A.ld + j], A.arc[7 * A.ld + j], A.arc[8 * A.ld + j]);
    const double t1 = A.arc[9 * A.ld + j], t2 = A.arc[10 * A.ld + j];
    const D3 d = ref_dir(A, j);
    double ra, tha, pha, rc, thc, phc;
    sph(a, ra, tha, pha);
    sph(c, rc, thc, phc);
    const double rb = nrm(b), span = t2 - t1;
    const D3 ah = dvd(a, ra > 0.0 ? ra : 1.0);
    const D3 x = crs(ah, d);
    const double xn = nrm(x);
    const D3 bh = dvd(x, xn > 0.0 ? xn : 1.0);
    const D3 bd = dvd(b, rb > 0.0 ? rb : 1.0);
    const bool ok = ra >= A.rmin && ra <= 4.0 * A.rmax && rb >= 0.1 * A.rmin && rb <= A.rmax && rc <= A.rmax &&
                    t1 >= 0.0 && t1 < 2.0 * kPi && span >= 0.0 && span <= 2.0 * kPi && xn > 1e-6 &&
                    nrm(sub(bh, bd)) <= 1e-3;
    uint32_t *w = A.codes + 4 * j;
    if (ok) {
        Bits B;
        B.put(qlin(ra, A.rmin, 4.0 * A.rmax, kNr), kNr);
        B.put(qlin(tha, 0.0, kPi, kMth), kMth);
        B.put(qper(pha, kMph), kMph);
        B.put(qlin(rb, 0.1 * A.rmin, A.rmax, kNr), kNr);
        B.put(qlin(rc, 0.0, A.rmax, kNr), kNr);
        B.put(qlin(thc, 0.0, kPi, kMth), kMth);
        B.put(qper(phc, kMph), kMph);
        B.put(qper(t1, kNt), kNt);
        B.put(qlin(span, 0.0, 2.0 * kPi, kNt), kNt);
        w[0] = (uint32_t)B.lo;
        w[1] = (uint32_t)(B.lo >> 32);
        w[2] = (uint32_t)B.hi;
        w[3] = (uint32_t)(B.hi >> 32);
    } else {
        const unsigned long long slot = atomicAdd(A.fb_n, 1ull);
        atomicOr(&A.mask[j >> 5], 1u << (j & 31));
        if ((int64_t)slot < A.fb_cap)
            for (int f = 0; f < 11; ++f) A.fb[11 * (int64_t)slot + f] = A.arc[f * A.ld + j];
        w[0] = (uint32_t)slot;
        w[1] = (uint32_t)(slot >> 32);
        w[2] = 0;
        w[3] = 0;
    }
}

__global__ void k_arc_decode(CodecArgs A)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= A.E) return;
    const uint32_t *w = A.codes + 4 * j;
    float *o = A.out;
    const int64_t L = A.ld_out;
    if ((A.mask[j >> 5] >> (j & 31)) & 1u) {
        const int64_t slot = (int64_t)((unsigned long long)w[0] | ((unsigned long long)w[1] << 32));
        for (int f = 0; f < 11; ++f) o[f * L + j] = slot < A.fb_cap ? A.fb[11 * slot + f] : 0.f;
        return;
    }
    Bits B;
    B.lo = (unsigned long long)w[0] | ((unsigned long long)w[1] << 32);
    B.hi = (unsigned long long)w[2] | ((unsigned long long)w[3] << 32);
    const uint32_t qra = B.get(kNr), qtha = B.get(kMth), qpha = B.get(kMph), qrb = B.get(kNr);
    const uint32_t qrc = B.get(kNr), qthc = B.get(kMth), qphc = B.get(kMph), qt1 = B.get(kNt), qsp = B.get(kNt);
    const D3 a = cart(dlin(qra, A.rmin, 4.0 * A.rmax, kNr), dlin(qtha, 0.0, kPi, kMth), dper(qpha, kMph));
    const D3 c = cart(dlin(qrc, 0.0, A.rmax, kNr), dlin(qthc, 0.0, kPi, kMth), dper(qphc, kMph));
    const double an = nrm(a);
    const D3 ah = dvd(a, an > 1e-300 ? an : 1e-300);
    const D3 d = ref_dir(A, j);
    const D3 x = crs(ah, d);
    const double xn = nrm(x);
    const D3 b = scl(dvd(x, xn > 0.0 ? xn : 1.0), dlin(qrb, 0.1 * A.rmin, A.rmax, kNr));
    const double t1 = dper(qt1, kNt);
    const double t2 = t1 + dlin(qsp, 0.0, 2.0 * kPi, kNt);
    const double v[11] = {c.x, c.y, c.z, a.x, a.y, a.z, b.x, b.y, b.z, t1, t2};
    for (int f = 0; f < 11; ++f) o[f * L + j] = (float)v[f];
}

}  // namespace

hipError_t launch_arc_codec(const Inputs &in, const Work &w, bool encode, const float *arc, const uint32_t *u32,
                            int64_t E, int64_t ld, double rmin, double rmax, uint32_t *codes, uint32_t *mask,
                            float *fb, int64_t fb_cap, unsigned long long *fb_n, float *out, int64_t ld_out,
                            hipStream_t st)
{
    if (E == 0) return hipSuccess;
    CodecArgs A;
    A.in = in;
    A.w = w;
    A.arc = arc;
    A.u32 = u32;
    A.E = E;
    A.ld = ld;
    A.rmin = rmin;
    A.rmax = rmax;
    A.codes = codes;
    A.mask = mask;
    A.fb = fb;
    A.fb_cap = fb_cap;
    A.fb_n = fb_n;
    A.out = out;
    A.ld_out = ld_out;
    const unsigned g = (unsigned)((E + 255) / 256);
    if (encode) k_arc_encode<<<g, 256, 0, st>>>(A);
    else k_arc_decode<<<g, 256, 0, st>>>(A);
    return hipGetLastError();
}

}  // namespace lm
