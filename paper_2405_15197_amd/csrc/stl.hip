// Binary STL output of an indexed triangle mesh held on the device, through
// an asynchronous device -> host -> disk pipeline (the paper's output stage,
// Sec. 4.2.2: batches sized by the I/O buffer, Eq. 6 with 50-byte triangle
// records, transfers overlapped with computation).  Here the triangulation
// itself runs on the GPU, so what crosses PCIe is the finished STL records:
// the device encodes chunk i (triangle soup with unit normals) while chunk
// i-1 is copied to pinned host memory on a second stream and written to the
// file by the calling thread.  (Four writer threads per chunk measured no
// faster: the pipeline is bound by the disk.)
#include <errno.h>
#include <fcntl.h>
#include <stdint.h>
#include <string.h>
#include <time.h>
#include <unistd.h>

#include <hip/hip_runtime.h>

#include "../../include/latmesh.h"

namespace {

constexpr int kStlBlock = 256;        // triangles per block
constexpr int kStlRec = 50;           // bytes per STL triangle record
constexpr int kStlWords = kStlBlock * kStlRec / 4;

// One block encodes 256 triangles into LDS (25 half-words each: normal,
// three vertices, a zero attribute word) and writes the 12,800-byte image
// with whole-word stores.  Indices outside [0, M) give a zero triangle and
// raise *bad.
__global__ void __launch_bounds__(kStlBlock) k_stl_encode(const float *xyz, int64_t M, const int32_t *tri,
                                                          int64_t t0, int64_t nt, uint32_t *out, int *bad)
{
    __shared__ uint32_t img[kStlWords];
    uint16_t *h = (uint16_t *)img;
    const int64_t base = (int64_t)blockIdx.x * kStlBlock;
    const int i = threadIdx.x;
    const int64_t t = base + i;
    if (t < nt) {
        const int64_t g = t0 + t;
        const int32_t id[3] = {tri[3 * g], tri[3 * g + 1], tri[3 * g + 2]};
        float v[9];
        bool ok = true;
#pragma unroll
        for (int c = 0; c < 3; ++c) ok = ok && id[c] >= 0 && (int64_t)id[c] < M;
        if (ok) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[3 * c] = xyz[3 * (int64_t)id[c]];
                v[3 * c + 1] = xyz[3 * (int64_t)id[c] + 1];
                v[3 * c + 2] = xyz[3 * (int64_t)id[c] + 2];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 9; ++c) v[c] = 0.f;
            atomicOr(bad, 1);
        }
        // facet normal: the unit normal of (v1 - v0) x (v2 - v0), zero for a
        // degenerate triangle
        const float e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
        const float e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
        float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
        const float len = sqrtf(nx * nx + ny * ny + nz * nz);
        const float inv = len > 0.f ? 1.f / len : 0.f;
        nx *= inv;
        ny *= inv;
        nz *= inv;
        const float f[12] = {nx, ny, nz, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8]};
        uint16_t *r = h + 25 * i;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const uint32_t b = __float_as_uint(f[c]);
            r[2 * c] = (uint16_t)(b & 0xffffu);
            r[2 * c + 1] = (uint16_t)(b >> 16);
        }
        r[24] = 0;
    }
    __syncthreads();
    const int64_t n = nt - base < kStlBlock ? nt - base : kStlBlock;
    const int bytes = (int)n * kStlRec;  // even
    uint32_t *dst = out + base * kStlRec / 4;  // base is a multiple of 256: word aligned
    for (int w = i; w < bytes / 4; w += kStlBlock) dst[w] = img[w];
    if ((bytes & 3) && i == 0) ((uint16_t *)dst)[bytes / 2 - 1] = h[bytes / 2 - 1];
}

double now_s()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int pwrite_all(int fd, const void *p, size_t n, int64_t off)
{
    const char *c = (const char *)p;
    while (n > 0) {
        const ssize_t w = ::pwrite(fd, c, n, (off_t)off);
        if (w < 0) {
            if (errno == EINTR) continue;
            return LM_ERR_IO;
        }
        c += w;
        off += w;
        n -= (size_t)w;
    }
    return LM_OK;
}

// Everything the pipeline allocates, released on every return path once
// both streams have drained (an error can leave a chunk in flight).
struct StlRes {
    hipStream_t st = nullptr;
    uint32_t *dev[2] = {nullptr, nullptr};
    uint8_t *host[2] = {nullptr, nullptr};
    int *bad = nullptr;
    hipStream_t copy = nullptr;
    hipEvent_t ev[8] = {};  // enc start / enc done / copy start / copy done, per buffer
    int fd = -1;
    ~StlRes()
    {
        if (copy) (void)hipStreamSynchronize(copy);
        if (dev[0] || bad) (void)hipStreamSynchronize(st);
        for (int b = 0; b < 2; ++b) {
            if (dev[b]) (void)hipFree(dev[b]);
            if (host[b]) (void)hipHostFree(host[b]);
        }
        if (bad) (void)hipFree(bad);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (copy) (void)hipStreamDestroy(copy);
        if (fd >= 0) ::close(fd);
    }
};

#define STLCHK(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) return LM_ERR_HIP;   \
    } while (0)

}  // namespace

extern "C" {

int lm_write_stl(const float *d_mesh_xyz, int64_t n_mesh_vertices, const int32_t *d_tri, int64_t n_triangles,
                 const char *path, int64_t chunk_bytes, int flags, void *stream, lm_stl_stats *stats)
{
    const double t_start = now_s();
    if (n_mesh_vertices < 0 || n_triangles < 0 || chunk_bytes < (int64_t)kStlBlock * kStlRec)
        return LM_ERR_INVALID_ARG;
    if (n_triangles > 0 && (!d_tri || !d_mesh_xyz)) return LM_ERR_INVALID_ARG;
    if (n_triangles > (int64_t)0xffffffffLL) return LM_ERR_UNSUPPORTED;  // the count field is 32 bits
    // chunk: whole blocks of 256 triangles
    int64_t chunk = chunk_bytes / kStlRec / kStlBlock * kStlBlock;
    if (chunk > n_triangles) chunk = (n_triangles + kStlBlock - 1) / kStlBlock * kStlBlock;
    if (chunk < kStlBlock) chunk = kStlBlock;
    const int64_t n_chunks = (n_triangles + chunk - 1) / chunk;
    const size_t buf_bytes = (size_t)chunk * kStlRec;
    hipStream_t st = (hipStream_t)stream;
    StlRes R;
    R.st = st;
    if (path) {
        R.fd = ::open(path, O_WRONLY | O_CREAT | O_TRUNC, 0644);
        if (R.fd < 0) return LM_ERR_IO;
    }
    // 80-byte header (not starting with "solid") and the triangle count
    uint8_t head[84];
    memset(head, ' ', 80);
    const char *tag = "binary STL, latmesh arc-subdivision triangulation";
    memcpy(head, tag, strlen(tag));
    const uint32_t cnt = (uint32_t)n_triangles;
    memcpy(head + 80, &cnt, 4);
    double write_s = 0.0;
    if (R.fd >= 0) {
        const double t0 = now_s();
        int rc = pwrite_all(R.fd, head, sizeof(head), 0);
        write_s += now_s() - t0;
        if (rc) return rc;
    }
    double enc_ms = 0.0, copy_ms = 0.0;
    if (n_chunks > 0) {
        STLCHK(hipMalloc((void **)&R.bad, sizeof(int)));
        STLCHK(hipMemsetAsync(R.bad, 0, sizeof(int), st));
        for (int b = 0; b < 2 && b < n_chunks; ++b) {
            STLCHK(hipMalloc((void **)&R.dev[b], buf_bytes));
            STLCHK(hipHostMalloc((void **)&R.host[b], buf_bytes, hipHostMallocDefault));
        }
        STLCHK(hipStreamCreateWithFlags(&R.copy, hipStreamNonBlocking));
        for (hipEvent_t &e : R.ev) STLCHK(hipEventCreate(&e));
        auto ev = [&](int b, int k) { return R.ev[4 * b + k]; };
        // chunk c: encode on the caller's stream into dev[c % 2] (after the
        // copy of chunk c - 2 out of it), copy to host[c % 2] on the copy
        // stream; the host writes chunk c - 1 while chunk c is in flight
        auto issue = [&](int64_t c) -> int {
            const int b = (int)(c & 1);
            const int64_t t0 = c * chunk, nt = n_triangles - t0 < chunk ? n_triangles - t0 : chunk;
            if (c >= 2) STLCHK(hipStreamWaitEvent(st, ev(b, 3), 0));
            STLCHK(hipEventRecord(ev(b, 0), st));
            k_stl_encode<<<(unsigned)((nt + kStlBlock - 1) / kStlBlock), kStlBlock, 0, st>>>(
                d_mesh_xyz, n_mesh_vertices, d_tri, t0, nt, R.dev[b], R.bad);
            STLCHK(hipGetLastError());
            STLCHK(hipEventRecord(ev(b, 1), st));
            STLCHK(hipStreamWaitEvent(R.copy, ev(b, 1), 0));
            STLCHK(hipEventRecord(ev(b, 2), R.copy));
            STLCHK(hipMemcpyAsync(R.host[b], R.dev[b], (size_t)nt * kStlRec, hipMemcpyDeviceToHost, R.copy));
            STLCHK(hipEventRecord(ev(b, 3), R.copy));
            return LM_OK;
        };
        auto drain = [&](int64_t c) -> int {
            const int b = (int)(c & 1);
            const int64_t t0 = c * chunk, nt = n_triangles - t0 < chunk ? n_triangles - t0 : chunk;
            STLCHK(hipEventSynchronize(ev(b, 3)));
            float ms = 0.f;
            STLCHK(hipEventElapsedTime(&ms, ev(b, 0), ev(b, 1)));
            enc_ms += ms;
            STLCHK(hipEventElapsedTime(&ms, ev(b, 2), ev(b, 3)));
            copy_ms += ms;
            if (R.fd >= 0) {
                const double w0 = now_s();
                int rc = pwrite_all(R.fd, R.host[b], (size_t)nt * kStlRec, 84 + t0 * kStlRec);
                write_s += now_s() - w0;
                if (rc) return rc;
            }
            return LM_OK;
        };
        int rc = issue(0);
        if (rc) return rc;
        for (int64_t c = 1; c < n_chunks; ++c) {
            // host[c % 2] held chunk c - 2, written out by the previous drain
            if ((rc = issue(c))) return rc;
            if ((rc = drain(c - 1))) return rc;
        }
        if ((rc = drain(n_chunks - 1))) return rc;
        int bad = 0;
        STLCHK(hipMemcpyAsync(&bad, R.bad, sizeof(int), hipMemcpyDeviceToHost, st));
        STLCHK(hipStreamSynchronize(st));
        if (bad) return LM_ERR_INVALID_ARG;
    }
    if (R.fd >= 0 && (flags & LM_STL_FSYNC)) {
        const double w0 = now_s();
        if (::fsync(R.fd) != 0) return LM_ERR_IO;
        write_s += now_s() - w0;
    }
    if (R.fd >= 0) {
        const int fd = R.fd;
        R.fd = -1;
        if (::close(fd) != 0) return LM_ERR_IO;
    }
    if (stats) {
        stats->n_triangles = n_triangles;
        stats->n_bytes = 84 + (int64_t)kStlRec * n_triangles;
        stats->n_chunks = n_chunks;
        stats->chunk_triangles = chunk;
        stats->seconds = now_s() - t_start;
        stats->encode_ms = enc_ms;
        stats->copy_ms = copy_ms;
        stats->write_s = write_s;
    }
    return LM_OK;
}

}  // extern "C"
