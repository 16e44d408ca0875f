// Device-side generation of the seeded BCC lattice (the same arrays as
// latgen.bcc, bit for bit): for lattices too large to build on the host.
// Input generation only; none of the meshing arithmetic.
//
// Every value is computed in FP64 in the order latgen uses and rounded once
// to FP32.  This file must be compiled without floating-point contraction
// (-ffp-contract=off) so that no multiply-add is fused.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ inline uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// latgen.uniform(seed, id, field)
__device__ inline double uniform(uint64_t seed, uint64_t id, uint64_t field)
{
    const uint64_t k = splitmix64(seed * 0x100000001B3ull + field);
    uint64_t z = splitmix64(id ^ k);
    z = splitmix64(z + (field + 1));
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

struct Spec {
    int64_t n;       // cells per side
    int order;       // 0: all corners, then all centres; 1: layer by layer
    int kind;        // 0: constant, 1: uniform(lo, hi), 2: rel(base, frac)
    double a, b;     // constant: a; uniform: lo, hi - lo; rel: base, frac
    double jitter, cell;
    uint64_t seed;
};

__global__ void k_bcc_nodes(Spec P, float *x, float *y, float *z, float *r)
{
    const int64_t m = P.n + 1, nc = m * m * m, N = nc + P.n * P.n * P.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double p[3];
    if (P.order == 0) {
        if (i < nc) {
            p[0] = (double)(i % m);
            p[1] = (double)((i / m) % m);
            p[2] = (double)(i / (m * m));
        } else {
            const int64_t c = i - nc;
            p[0] = (double)(c % P.n) + 0.5;
            p[1] = (double)((c / P.n) % P.n) + 0.5;
            p[2] = (double)(c / (P.n * P.n)) + 0.5;
        }
    } else {
        // layer l: its m^2 corners, then (below the top layer) the n^2
        // centres just above it
        const int64_t B = m * m + P.n * P.n, l = i / B, r = i % B;
        if (r < m * m) {
            p[0] = (double)(r % m);
            p[1] = (double)(r / m);
            p[2] = (double)l;
        } else {
            const int64_t c = r - m * m;
            p[0] = (double)(c % P.n) + 0.5;
            p[1] = (double)(c / P.n) + 0.5;
            p[2] = (double)l + 0.5;
        }
    }
    for (int d = 0; d < 3; ++d) {
        double q = p[d] * P.cell;
        double j = 0.0;
        if (P.jitter != 0.0) j = (2.0 * uniform(P.seed, (uint64_t)i, (uint64_t)d) - 1.0) * P.jitter * P.cell;
        q = q + j;
        (d == 0 ? x : d == 1 ? y : z)[i] = (float)q;
    }
    double rad;
    if (P.kind == 0) {
        rad = P.a * P.cell;
    } else {
        const double u = uniform(P.seed, (uint64_t)i, 3);
        rad = P.kind == 1 ? (P.a + P.b * u) * P.cell : P.a * (1.0 + P.b * (2.0 * u - 1.0)) * P.cell;
    }
    r[i] = (float)rad;
}

__global__ void k_bcc_struts(Spec P, int32_t *sa, int32_t *sb)
{
    const int64_t m = P.n + 1, n3 = P.n * P.n * P.n;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= 8 * n3) return;
    const int64_t c = s >> 3;
    const int corner = (int)(s & 7);
    const int64_t ci = c % P.n, cj = (c / P.n) % P.n, ck = c / (P.n * P.n);
    const int64_t di = corner & 1, dj = (corner >> 1) & 1, dk = (corner >> 2) & 1;
    if (P.order == 0) {
        sa[s] = (int32_t)((ci + di) + m * ((cj + dj) + m * (ck + dk)));
        sb[s] = (int32_t)(m * m * m + c);
    } else {
        const int64_t B = m * m + P.n * P.n;
        sa[s] = (int32_t)((ck + dk) * B + (ci + di) + m * (cj + dj));
        sb[s] = (int32_t)(ck * B + m * m + ci + P.n * cj);
    }
}

}  // namespace

extern "C" {

// BCC lattice of n^3 cells into device arrays x, y, z, r [(n+1)^3 + n^3] and
// sa, sb [8 n^3].  radius_kind 0: a (constant), 1: U[a, a + b], 2: a (1 +
// b U[-1, 1]); all times cell.  order 0: corners then centres; 1: layer by
// layer (latgen.bcc's order="layer").  Returns 0 or a HIP error code.
int lg_bcc(int64_t n, int order, int radius_kind, double a, double b, double jitter, uint64_t seed, double cell, float *x,
           float *y, float *z, float *r, int32_t *sa, int32_t *sb, void *stream)
{
    Spec P{n, order, radius_kind, a, b, jitter, cell, seed};
    const int64_t m = n + 1, N = m * m * m + n * n * n, S = 8 * n * n * n;
    hipStream_t st = (hipStream_t)stream;
    if (N > 0) k_bcc_nodes<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(P, x, y, z, r);
    if (S > 0) k_bcc_struts<<<(unsigned)((S + 255) / 256), 256, 0, st>>>(P, sa, sb);
    return (int)hipGetLastError();
}

}  // extern "C"
