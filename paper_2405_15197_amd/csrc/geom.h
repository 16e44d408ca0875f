// Node-local geometry shared by the meta-meshing and adjoint kernels:
// scalar helpers over float / double (and the adjoint's dual numbers),
// 3-vectors, the strut table of a node and its seam conics (Sec. 4.1,
// Sec. 4.3.1, Eq. 7).  Not installed.
#pragma once

#include "common.h"

namespace lm {
namespace geo {

// ---------------------------------------------------------------------------
// scalar helpers (float / double)

__device__ inline float m_sqrt(float x) { return sqrtf(x); }
__device__ inline double m_sqrt(double x) { return sqrt(x); }
__device__ inline float m_abs(float x) { return fabsf(x); }
__device__ inline double m_abs(double x) { return fabs(x); }
__device__ inline float m_atan2(float y, float x) { return atan2f(y, x); }
__device__ inline double m_atan2(double y, double x) { return atan2(y, x); }
// quotient for keys that only order angles (a few ulp suffice)
__device__ inline float m_qdiv(float x, float y) { return __fdividef(x, y); }
__device__ inline double m_qdiv(double x, double y) { return x / y; }
__device__ inline float m_floor(float x) { return floorf(x); }
__device__ inline double m_floor(double x) { return floor(x); }
__device__ inline float m_max(float a, float b) { return fmaxf(a, b); }
__device__ inline double m_max(double a, double b) { return fmax(a, b); }
__device__ inline void m_sincos(float t, float *s, float *c) { sincos_f32(t, s, c); }
__device__ inline void m_sincos(double t, double *s, double *c) { sincos(t, s, c); }

template <typename T>
struct Cst {
    static constexpr T two_pi = (T)6.283185307179586476925286766559;
    static constexpr T pi = (T)3.1415926535897932384626433832795;
    static constexpr T inv_two_pi = (T)0.15915494309189533576888376337251;
};

template <typename T>
struct V3 {
    T x, y, z;
};
template <typename T>
__device__ inline V3<T> v3(T x, T y, T z) { return V3<T>{x, y, z}; }
template <typename T>
__device__ inline V3<T> operator+(V3<T> a, V3<T> b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
template <typename T>
__device__ inline V3<T> operator-(V3<T> a, V3<T> b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
template <typename T>
__device__ inline V3<T> operator*(V3<T> a, T s) { return v3(a.x * s, a.y * s, a.z * s); }
template <typename T>
__device__ inline T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ inline V3<T> cross(V3<T> a, V3<T> b)
{
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <typename T>
__device__ inline V3<T> zero3() { return v3((T)0, (T)0, (T)0); }

template <typename T>
struct SL {
    T gx, gy, gz, h;   // P_m(w) = g . w - h
    T ex, ey, ez, sig; // unit direction node -> far node, sigma
    T rx, ry, rz, kap; // strut frame r, kappa
    T qx, qy, qz, len; // strut frame q, length
    T sx, sy, sz;      // canonical strut direction (lower -> higher node id)
    int lower, sid, far;
};

template <typename T>
__device__ inline V3<T> gvec(const SL<T> &s) { return v3(s.gx, s.gy, s.gz); }

// Strut table entry of incident strut (centre cf, radius rf) at the node
// (centre cen, radius rho): e, sigma, kappa, P_m = g . w - h, the length and
// the canonical strut frame from the lower to the higher node id (both ends
// compute it from the same two input positions).  bad: zero length or
// |sigma| >= 1 (then the entry is computed with L = 1, sigma = 0).
template <typename T>
__device__ inline SL<T> strut_entry(V3<T> cen, T rho, V3<T> cf, T rf, int lower, bool &bad)
{
    SL<T> s;
    V3<T> d = cf - cen;
    T L = m_sqrt(dot(d, d));
    T sig = (rho - rf) / L;
    bad = !(L > (T)0) || !(m_abs(sig) < (T)1);
    if (bad) {
        L = (T)1;
        sig = (T)0;
    }
    T kap = m_sqrt(((T)1 - sig) * ((T)1 + sig));
    V3<T> e = d * ((T)1 / L);
    s.ex = e.x; s.ey = e.y; s.ez = e.z; s.sig = sig; s.kap = kap; s.len = L;
    s.gx = e.x / kap; s.gy = e.y / kap; s.gz = e.z / kap;
    s.h = rho * sig / kap;
    s.lower = lower;
    V3<T> clo = lower ? cen : cf;
    V3<T> chi = lower ? cf : cen;
    V3<T> es = chi - clo;
    es = es * ((T)1 / m_sqrt(dot(es, es)));
    s.sx = es.x; s.sy = es.y; s.sz = es.z;
    // reference axis: the coordinate axis of smallest |e_i| (lowest index on ties)
    T ax = m_abs(es.x), ay = m_abs(es.y), az = m_abs(es.z);
    int j = 0;
    T am = ax;
    if (ay < am) { j = 1; am = ay; }
    if (az < am) { j = 2; }
    V3<T> axis = v3((T)(j == 0 ? 1 : 0), (T)(j == 1 ? 1 : 0), (T)(j == 2 ? 1 : 0));
    V3<T> rr = cross(es, axis);
    rr = rr * ((T)1 / m_sqrt(dot(rr, rr)));
    V3<T> qq = cross(es, rr);
    s.rx = rr.x; s.ry = rr.y; s.rz = rr.z;
    s.qx = qq.x; s.qy = qq.y; s.qz = qq.z;
    return s;
}

// ---------------------------------------------------------------------------
// conics

template <typename T>
struct Con {
    V3<T> o, a, b;
};

template <typename T>
__device__ inline V3<T> conic_at(const Con<T> &C, T t)
{
    T s, c;
    m_sincos(t, &s, &c);
    return C.o + C.a * s + C.b * c;
}

// Conic (p, q) of the node.  Returns false if the section is not an ellipse.
template <typename T>
__device__ bool conic_of(const SL<T> *S, T rho, int p, int q, Con<T> &C)
{
    if (p == 0) {
        const SL<T> &s = S[q];
        T rad = rho * s.kap;
        C.o = v3(s.ex, s.ey, s.ez) * (rho * s.sig);
        C.a = v3(s.qx, s.qy, s.qz) * rad;
        C.b = v3(s.rx, s.ry, s.rz) * rad;
        return true;
    }
    const SL<T> &P = S[p], &Q = S[q];
    V3<T> gp = gvec(P);
    V3<T> n = gp - gvec(Q);
    T nn = m_sqrt(dot(n, n));
    V3<T> nh = n * ((T)1 / nn);
    T d0 = (P.h - Q.h) / nn;            // plane: nh . w = d0
    T gpn = dot(gp, nh);
    T epn = m_abs(gpn * P.kap);         // |e_p . nh|
    T as = m_abs(P.sig);
    T om = (epn - as) * (epn + as) / (P.kap * P.kap); // 1 - |in-plane g_p|^2
    if (!(om > (T)0)) return false;
    V3<T> gam = gp - nh * gpn;          // in-plane part of g_p: major axis direction
    T gl = m_sqrt(dot(gam, gam));
    V3<T> u1;
    // Below a relative 1e-4 the in-plane part is rounding (exactly opposite
    // struts make the section a circle) and its direction means nothing: any
    // in-plane axis parametrises the (almost) circle.
    if (gl > (T)1e-4 * m_sqrt(dot(gp, gp))) {
        u1 = gam * ((T)1 / gl);
        // gam is a small difference when the plane is nearly perpendicular
        // to the axis; keep u1 exactly in the plane (its in-plane rotation
        // error only reparametrises an almost circular ellipse)
        u1 = u1 - nh * dot(u1, nh);
        u1 = u1 * ((T)1 / m_sqrt(dot(u1, u1)));
    } else {
        V3<T> t = m_abs(nh.x) < (T)0.9 ? v3((T)1, (T)0, (T)0) : v3((T)0, (T)1, (T)0);
        u1 = cross(nh, t);
        u1 = u1 * ((T)1 / m_sqrt(dot(u1, u1)));
    }
    // in-plane coordinates w = d0 nh + al u1 + be u2:
    //   (1 - gl^2) al^2 - 2 gl k0 al + be^2 = rho^2 - d0^2 + k0^2,
    // k0 = P_p at the foot point d0 nh; complete the square.
    T k0 = d0 * gpn - P.h;
    T al0 = gl * k0 / om;
    T R2 = rho * rho - d0 * d0 + k0 * k0 / om;
    T R = m_sqrt(m_max(R2, (T)0));
    C.o = nh * d0 + u1 * al0;
    C.a = u1 * (R / m_sqrt(om));
    C.b = cross(u1, nh) * R;
    return true;
}

}  // namespace geo
}  // namespace lm
