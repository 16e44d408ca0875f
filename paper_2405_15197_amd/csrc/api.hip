// Host side of the C ABI declared in include/latmesh.h.
#include <new>
#include <utility>
#include <string.h>
#include <vector>

#include "../../include/latmesh.h"
#include "common.h"

// Phases timed with HIP events when profiling is on (lm_set_profiling).
enum Phase { PH_PREPARE, PH_NODE32, PH_NODE64, PH_SIZES, PH_EXPAND, PH_ZIP, PH_LOSS, PH_BACKWARD, PH_N };

struct lm_plan {
    lm::Inputs in;
    lm::Work w;
    hipStream_t st;
    void *ws;       // one allocation for the fixed-size workspace
    int64_t rec_alloc_words;  // words allocated for node records
    // sink mode (allocated at the first lm_forward_sink)
    int32_t *sk_mark = nullptr;     // [N] epoch of the last chunk listing the node
    int32_t *sk_lists = nullptr;    // [kClasses][N] chunk node lists
    int32_t *sk_cnt = nullptr;      // [4] list sizes, then the strut count
    int64_t *sk_info = nullptr;     // [8] class sizes / starts for the node kernel
    int32_t *sk_struts = nullptr;   // [sk_struts_cap] struts owned by the chunk
    int64_t sk_struts_cap = 0;
    unsigned long long *sk_slots = nullptr;
    int32_t sk_epoch = 0;
    // second record slot (re-subdivision): records, node record index, bump
    // counters; base_slot says where the meta-mesh of the last count is
    uint32_t *alt_rec = nullptr;
    int64_t alt_rec_words = 0;
    int64_t *alt_node_rec = nullptr;
    unsigned long long *alt_rec_top = nullptr;
    int base_slot = 0;
    // the allocations behind the second node record index and counters (the
    // pointers above swap with the workspace's own at every switch), and the
    // redo lists [N] and their counters [8]
    void *alt_index_mem = nullptr;
    int32_t *redo = nullptr;
    int32_t *redo_cnt = nullptr;
    unsigned long long *codec_ctr = nullptr;  // fallback counter of lm_arc_encode
    void *grad_mem = nullptr;                 // adjoint scratch (loss terms and partials per node / half-edge)
    int schedule = LM_SCHEDULE_WAVE;          // FP32 node pass of lm_count / lm_forward
    void *thread_scratch = nullptr;           // per-node scratch of the thread-centric pass
    int k;          // resolution of the last count (0: none)
    float kappa_max;// FP32 -> FP64 hand-over threshold
    lm_totals last; // totals of the last lm_count
    bool last_on_host = false;  // `last` describes the current mesh (lm_count ran last)
    bool profiling;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
    std::vector<hipEvent_t> pool;
};

__global__ void lm_k_status_u8(const int32_t *s, uint8_t *d, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (uint8_t)s[i];
}

namespace {

hipEvent_t take_event(lm_plan *P)
{
    if (!P->pool.empty()) {
        hipEvent_t e = P->pool.back();
        P->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event pair around one phase when profiling.
struct PhaseTimer {
    lm_plan *P;
    int ph;
    hipEvent_t a = nullptr, b = nullptr;
    PhaseTimer(lm_plan *P_, int ph_) : P(P_), ph(ph_)
    {
        if (P->profiling) {
            a = take_event(P);
            b = take_event(P);
            if (a) (void)hipEventRecord(a, P->st);
        }
    }
    ~PhaseTimer()
    {
        if (a && b) {
            (void)hipEventRecord(b, P->st);
            P->ev.push_back({ph, {a, b}});
        }
    }
};

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return LM_ERR_HIP;    \
    } while (0)

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Carve the workspace; with base == nullptr only the size is computed.
size_t carve(lm::Work &w, char *base, int64_t N, int64_t S)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const int64_t H = 2 * S;
    w.node4 = (float4 *)take(sizeof(float4) * (N + 1));
    w.row = (int64_t *)take(sizeof(int64_t) * (N + 1));
    w.he = (int2 *)take(sizeof(int2) * (H + 1));
    w.deg = (int32_t *)take(sizeof(int32_t) * (N + 1));
    w.strut_he = (int64_t *)take(sizeof(int64_t) * (H + 1));
    w.node_cnt = (int32_t *)take(sizeof(int32_t) * lm::kNodeCols * (N + 1));
    w.node_off = (int64_t *)take(sizeof(int64_t) * lm::kNodeScanCols * (N + 1));
    w.he_len = (int32_t *)take(sizeof(int32_t) * (H + 1));
    w.he_loop = (int64_t *)take(sizeof(int64_t) * (H + 1));
    w.he_rot = (int32_t *)take(sizeof(int32_t) * (H + 1));
    w.band_cnt = (int32_t *)take(sizeof(int32_t) * (S + 1));
    w.band_off = (int64_t *)take(sizeof(int64_t) * (S + 1));
    int64_t tl = lm::scan_tmp_needed(N, lm::kNodeScanCols);
    int64_t t2 = lm::scan_tmp_needed(S, 1);
    if (t2 > tl) tl = t2;
    w.scan_tmp = (int64_t *)take(sizeof(int64_t) * tl);
    w.scan_tmp_len = tl;
    w.flags = (int32_t *)take(sizeof(int32_t) * 4);
    w.totals = (int64_t *)take(sizeof(int64_t) * 16);
    w.fb_list = (int32_t *)take(sizeof(int32_t) * (N + 1));
    w.node_rec = (int64_t *)take(sizeof(int64_t) * (N + 1));
    w.rec_top = (unsigned long long *)take(sizeof(unsigned long long) * lm::kRecRegions);
    w.queue = (int32_t *)take(sizeof(int32_t) * (N + 1));
    w.cls_info = (int64_t *)take(sizeof(int64_t) * 8);
    w.work_ctr = (int32_t *)take(sizeof(int32_t) * 4);
    w.node_k = nullptr;
    w.loss_node = nullptr;
    w.grad_node = nullptr;
    w.grad_he = nullptr;
    return off;
}

lm::FillOut to_fill(const lm_outputs *o)
{
    lm::FillOut f;
    f.mesh_xyz = o->d_mesh_xyz;
    f.tri = o->d_tri;
    f.cap_mesh = o->cap_mesh_vertices;
    f.cap_tri = o->cap_triangles;
    f.vert_name = o->d_vert_name;
    f.vert_xyz = o->d_vert_xyz;
    f.cap_vert = o->cap_vertices;
    f.arc_f32 = o->d_arc_f32;
    f.arc_u32 = o->d_arc_u32;
    f.cap_arc = o->cap_arcs;
    if (!f.vert_name || !f.vert_xyz) {
        f.vert_name = nullptr;
        f.vert_xyz = nullptr;
    }
    if (!f.arc_f32 || !f.arc_u32) {
        f.arc_f32 = nullptr;
        f.arc_u32 = nullptr;
    }
    return f;
}

// Count pass: per-node meta-meshing and counts, band counts, prefix sums,
// device totals (and capacity flags when out != nullptr).
// Node pass (meta-meshing at k, or with src_rec set the re-subdivision of
// the meta-mesh in those records) into the records of w, then band counts,
// prefix sums and device totals.
int run_count(lm_plan *P, int k, const lm::FillOut *out, const lm::Work &w, const uint32_t *src_rec = nullptr,
              const int64_t *src_node_rec = nullptr, int32_t *redo = nullptr, int32_t *redo_cnt = nullptr)
{
    const int64_t N = P->in.n_nodes, S = P->in.n_struts;
    // flags[0] (count / fill) and flags[2] (FP64 hand-over count)
    HIPCHK(hipMemsetAsync(w.flags, 0, sizeof(int32_t), P->st));
    HIPCHK(hipMemsetAsync(w.flags + 2, 0, sizeof(int32_t), P->st));
    HIPCHK(hipMemsetAsync(w.totals, 0, sizeof(int64_t) * 16, P->st));
    HIPCHK(hipMemsetAsync(w.rec_top, 0, sizeof(unsigned long long) * lm::kRecRegions, P->st));
    HIPCHK(hipMemsetAsync(w.work_ctr, 0, sizeof(int32_t) * 4, P->st));
    {
        PhaseTimer t(P, PH_NODE32);
        if (redo_cnt) HIPCHK(hipMemsetAsync(redo_cnt, 0, sizeof(int32_t) * 8, P->st));
        if (P->schedule == LM_SCHEDULE_THREAD && !src_rec) {
            if (!P->thread_scratch) HIPCHK(hipMalloc(&P->thread_scratch, lm::node_thread_scratch_bytes()));
            HIPCHK(lm::launch_node_thread(P->in, w, k, P->kappa_max, P->thread_scratch, P->st));
        } else {
            HIPCHK(lm::launch_node(P->in, w, k, P->kappa_max, 0, P->st, src_rec, src_node_rec, redo, redo_cnt));
        }
    }
    {
        PhaseTimer t(P, PH_NODE64);
        HIPCHK(lm::launch_node(P->in, w, k, P->kappa_max, 1, P->st, src_rec, src_node_rec));
    }
    PhaseTimer t(P, PH_SIZES);
    HIPCHK(lm::launch_band_count(P->in, w, P->st));
    HIPCHK(lm::launch_scan(w.node_cnt, w.node_off, N, lm::kNodeScanCols, N, N + 1, w.scan_tmp, w.scan_tmp_len,
                           P->st));
    HIPCHK(lm::launch_scan(w.band_cnt, w.band_off, S, 1, 0, 0, w.scan_tmp, w.scan_tmp_len, P->st));
    HIPCHK(lm::launch_totals(P->in, w, out, P->st));
    return LM_OK;
}

int read_totals(lm_plan *P, lm_totals *t, int32_t *flags_out)
{
    int64_t tv[16];
    int32_t fl[4];
    HIPCHK(hipMemcpyAsync(tv, P->w.totals, sizeof(tv), hipMemcpyDeviceToHost, P->st));
    HIPCHK(hipMemcpyAsync(fl, P->w.flags, sizeof(fl), hipMemcpyDeviceToHost, P->st));
    HIPCHK(hipStreamSynchronize(P->st));
    t->n_vertices = tv[0];
    t->n_arcs = tv[1];
    t->n_holes = tv[2];
    t->n_mesh_vertices = tv[3];
    t->n_triangles = tv[4];
    t->n_band_triangles = tv[5];
    t->n_fan_triangles = tv[6];
    t->n_record_bytes = tv[7];
    t->n_bad_nodes = tv[8];
    t->n_skipped_struts = tv[9];
    t->n_fp64_nodes = tv[10];
    *flags_out = fl[0] | fl[1];
    return LM_OK;
}

// Node-record space: at least `words` (rounded so the regions are equal and
// 16-byte aligned).  Synchronises the stream before replacing the buffer.
int ensure_rec(lm_plan *P, int64_t words)
{
    const int64_t unit = 4 * lm::kRecRegions;
    words = (words + unit - 1) / unit * unit;
    if (words <= P->w.rec_words) return LM_OK;
    HIPCHK(hipStreamSynchronize(P->st));
    if (P->w.rec) HIPCHK(hipFree(P->w.rec));
    P->w.rec = nullptr;
    P->w.rec_words = 0;
    HIPCHK(hipMalloc((void **)&P->w.rec, sizeof(uint32_t) * words));
    P->w.rec_words = words;
    return LM_OK;
}

// First guess of the record space at resolution k: per node the header and
// about 2 vertices, 3 arcs and a hole per incident strut; per half-edge a
// loop of about k samples.
int64_t rec_estimate(const lm_plan *P, int k)
{
    const int64_t N = P->in.n_nodes, H = 2 * P->in.n_struts;
    int64_t words = N * (lm::kRecHead + 4) + H * (2 * 4 + 3 * lm::kRecArcFields + 3 + 2 * (int64_t)(k + 4));
    return words + words / 8 + 4096;
}

int fill_common(lm_plan *P, int k, const lm::FillOut &f, const lm_outputs *out, const lm::Work &w)
{
    const int64_t N = P->in.n_nodes;
    {
        PhaseTimer t(P, PH_EXPAND);
        HIPCHK(lm::launch_expand(P->in, w, f, P->st));
    }
    {
        PhaseTimer t(P, PH_ZIP);
        HIPCHK(lm::launch_zip(P->in, w, f, k, P->st));
    }
    if (out->d_node_off)
        HIPCHK(hipMemcpyAsync(out->d_node_off, w.node_off, sizeof(int64_t) * lm::kNodeScanCols * (N + 1),
                              hipMemcpyDeviceToDevice, P->st));
    if (out->d_strut_off)
        HIPCHK(hipMemcpyAsync(out->d_strut_off, w.band_off, sizeof(int64_t) * (P->in.n_struts + 1),
                              hipMemcpyDeviceToDevice, P->st));
    if (out->d_node_status && N > 0) {
        // int32 status column -> uint8 (values fit in 8 bits)
        lm_k_status_u8<<<(unsigned)((N + 255) / 256), 256, 0, P->st>>>(
            w.node_cnt + (int64_t)lm::NC_STATUS * N, out->d_node_status, N);
        HIPCHK(hipGetLastError());
    }
    return LM_OK;
}

}  // namespace

extern "C" {

int lm_plan_create(lm_plan **plan, const lm_lattice *lat, void *stream)
{
    if (!plan) return LM_ERR_INVALID_ARG;
    *plan = nullptr;
    if (!lat || lat->n_nodes < 0 || lat->n_struts < 0) return LM_ERR_INVALID_ARG;
    if (lat->n_nodes > 0 && (!lat->d_x || !lat->d_y || !lat->d_z || !lat->d_radius)) return LM_ERR_INVALID_ARG;
    if (lat->n_struts > 0 && (!lat->d_strut_a || !lat->d_strut_b)) return LM_ERR_INVALID_ARG;
    // node and strut ids are int32; half-edge indices are int64
    if (lat->n_nodes >= ((int64_t)1 << 31) || lat->n_struts >= ((int64_t)1 << 31)) return LM_ERR_UNSUPPORTED;
    lm_plan *P = new (std::nothrow) lm_plan();
    if (!P) return LM_ERR_INTERNAL;
    P->st = (hipStream_t)stream;
    P->in.n_nodes = lat->n_nodes;
    P->in.n_struts = lat->n_struts;
    P->in.x = lat->d_x;
    P->in.y = lat->d_y;
    P->in.z = lat->d_z;
    P->in.r = lat->d_radius;
    P->in.sa = lat->d_strut_a;
    P->in.sb = lat->d_strut_b;
    size_t bytes = carve(P->w, nullptr, lat->n_nodes, lat->n_struts);
    if (hipMalloc(&P->ws, bytes) != hipSuccess) {
        delete P;
        return LM_ERR_HIP;
    }
    carve(P->w, (char *)P->ws, lat->n_nodes, lat->n_struts);
    P->w.rec = nullptr;
    P->w.rec_words = 0;
    P->kappa_max = 32.0f;
    P->profiling = false;
    int rc = LM_OK;
    int32_t fl = 0;
    if (hipMemsetAsync(P->w.flags, 0, sizeof(int32_t) * 4, P->st) != hipSuccess ||
        hipMemsetAsync(P->w.totals, 0, sizeof(int64_t) * 16, P->st) != hipSuccess ||
        lm::launch_prepare(P->in, P->w, P->st) != hipSuccess ||
        hipMemcpyAsync(&fl, P->w.flags + 1, sizeof(int32_t), hipMemcpyDeviceToHost, P->st) != hipSuccess ||
        hipStreamSynchronize(P->st) != hipSuccess) {
        rc = LM_ERR_HIP;
    } else if (fl & lm::DF_BADLAT) {  // set in flags[1]
        rc = LM_ERR_BAD_LATTICE;
    }
    if (rc != LM_OK) {
        (void)hipFree(P->ws);
        delete P;
        return rc;
    }
    *plan = P;
    return LM_OK;
}

int lm_count(lm_plan *P, int k, lm_totals *totals)
{
    if (!P || !totals || k < 3 || k > 4096) return LM_ERR_INVALID_ARG;
    int rc = LM_OK;
    if (P->w.rec_words == 0 && (rc = ensure_rec(P, rec_estimate(P, k)))) return rc;
    int32_t fl = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        if ((rc = run_count(P, k, nullptr, P->w))) return rc;
        if ((rc = read_totals(P, totals, &fl))) return rc;
        if (totals->n_mesh_vertices > 0x7fffffffLL) return LM_ERR_UNSUPPORTED;
        if (!(fl & lm::DF_RECCAP)) break;
        // the records did not fit: the totals hold the space they need
        if ((rc = ensure_rec(P, totals->n_record_bytes / 4 + totals->n_record_bytes / 64))) return rc;
    }
    if (fl & lm::DF_RECCAP) return LM_ERR_INTERNAL;
    P->k = k;
    P->base_slot = 0;
    P->last = *totals;
    P->last_on_host = true;
    return LM_OK;
}

int lm_fill(lm_plan *P, const lm_outputs *out)
{
    if (!P || !out || !out->d_mesh_xyz || !out->d_tri) return LM_ERR_INVALID_ARG;
    if (P->k == 0) return LM_ERR_STATE;
    const lm_totals &t = P->last;
    if (out->cap_mesh_vertices < t.n_mesh_vertices || out->cap_triangles < t.n_triangles) return LM_ERR_CAPACITY;
    lm::FillOut f = to_fill(out);
    if (f.vert_name && out->cap_vertices < t.n_vertices) return LM_ERR_CAPACITY;
    if (f.arc_f32 && out->cap_arcs < t.n_arcs) return LM_ERR_CAPACITY;
    if (P->base_slot != 0) return LM_ERR_STATE;  // re-subdivided since lm_count
    return fill_common(P, P->k, f, out, P->w);
}

int lm_forward(lm_plan *P, int k, const lm_outputs *out)
{
    if (!P || !out || !out->d_mesh_xyz || !out->d_tri || k < 3 || k > 4096) return LM_ERR_INVALID_ARG;
    lm::FillOut f = to_fill(out);
    int rc = LM_OK;
    if (P->w.rec_words == 0 && (rc = ensure_rec(P, rec_estimate(P, k)))) return rc;
    rc = run_count(P, k, &f, P->w);
    if (rc) return rc;
    P->k = k;
    P->base_slot = 0;
    P->last_on_host = false;
    return fill_common(P, k, f, out, P->w);
}

namespace {

// Scratch of lm_loss and lm_backward: per-node loss terms, per-node and
// per-half-edge adjoint partials (allocated at the first use).
int grad_alloc(lm_plan *P)
{
    if (P->grad_mem) return LM_OK;
    const int64_t N = P->in.n_nodes, H = 2 * P->in.n_struts;
    const size_t a = align_up(sizeof(double) * 3 * (N + 1)), b = align_up(sizeof(float) * 4 * (N + 1));
    const size_t c = align_up(sizeof(float) * 4 * (H + 1));
    HIPCHK(hipMalloc(&P->grad_mem, a + b + c));
    char *m = (char *)P->grad_mem;
    P->w.loss_node = (double *)m;
    P->w.grad_node = (float *)(m + a);
    P->w.grad_he = (float *)(m + a + b);
    return LM_OK;
}

}  // namespace

int lm_loss(lm_plan *P, const lm_outputs *out, const lm_loss_weights *w, double *d_terms, float *d_dl_dx)
{
    if (!P || !out || !w || !d_terms || !d_dl_dx || !out->d_mesh_xyz || !out->d_tri) return LM_ERR_INVALID_ARG;
    if (P->k == 0) return LM_ERR_STATE;
    // sizes known on the host (after lm_count): refuse small buffers before
    // any launch; otherwise the kernels check the device totals and skip
    // (lm_read_totals then reports LM_ERR_CAPACITY)
    if (P->last_on_host &&
        (out->cap_mesh_vertices < P->last.n_mesh_vertices || out->cap_triangles < P->last.n_triangles))
        return LM_ERR_CAPACITY;
    if (out->cap_mesh_vertices < 0 || out->cap_triangles < 0) return LM_ERR_INVALID_ARG;
    int rc = grad_alloc(P);
    if (rc) return rc;
    lm::FillOut f = to_fill(out);
    PhaseTimer t(P, PH_LOSS);
    HIPCHK(lm::launch_loss(P->in, P->w, f, make_float3(w->p0[0], w->p0[1], w->p0[2]), w->area, w->volume, w->sq_norm,
                           d_dl_dx, d_terms, P->st));
    return LM_OK;
}

int lm_backward(lm_plan *P, const float *d_dl_dx, float *d_grad_xyz, float *d_grad_radius)
{
    if (!P || !d_dl_dx || !d_grad_xyz || !d_grad_radius) return LM_ERR_INVALID_ARG;
    if (P->k == 0) return LM_ERR_STATE;
    int rc = grad_alloc(P);
    if (rc) return rc;
    PhaseTimer t(P, PH_BACKWARD);
    HIPCHK(lm::launch_backward(P->in, P->w, d_dl_dx, d_grad_xyz, d_grad_radius, P->st));
    return LM_OK;
}

namespace {

int sink_alloc(lm_plan *P)
{
    if (P->sk_mark) return LM_OK;
    const int64_t N = P->in.n_nodes;
    HIPCHK(hipMalloc((void **)&P->sk_mark, sizeof(int32_t) * (N + 1)));
    HIPCHK(hipMemsetAsync(P->sk_mark, 0, sizeof(int32_t) * (N + 1), P->st));
    HIPCHK(hipMalloc((void **)&P->sk_lists, sizeof(int32_t) * lm::kClasses * (N + 1)));
    HIPCHK(hipMalloc((void **)&P->sk_cnt, sizeof(int32_t) * 8));
    HIPCHK(hipMalloc((void **)&P->sk_info, sizeof(int64_t) * 8));
    HIPCHK(hipMalloc((void **)&P->sk_slots, sizeof(unsigned long long) * lm::sink_slots_words()));
    HIPCHK(hipMemsetAsync(P->sk_slots, 0, sizeof(unsigned long long) * lm::sink_slots_words(), P->st));
    return LM_OK;
}

}  // namespace

namespace {

// One node range in sink mode: its node list (range + higher-id halo) in
// valence classes (limits t16 / t32), the node pass, and the hashed
// outputs: to out_chunk through the slots, or per part (node_part set).
// k_avg sizes the first guess of the record space.
int sink_range(lm_plan *P, int k, int k_avg, int64_t n0, int64_t n1, int t16, int t32, uint64_t *out_chunk,
               const int32_t *node_part, uint64_t *out_parts, const int64_t *part_base)
{
    const int64_t N = P->in.n_nodes, S = P->in.n_struts;
    lm::Work &w = P->w;
    int rc = LM_OK;
    HIPCHK(hipMemsetAsync(P->sk_cnt, 0, sizeof(int32_t) * 8, P->st));
    if (++P->sk_epoch <= 0) {  // epochs wrapped: clear the marks
        HIPCHK(hipMemsetAsync(P->sk_mark, 0, sizeof(int32_t) * (N + 1), P->st));
        P->sk_epoch = 1;
    }
    {
        PhaseTimer t(P, PH_SIZES);
        HIPCHK(lm::launch_chunk_list(w, n0, n1, P->sk_mark, P->sk_epoch, P->sk_lists, N + 1, P->sk_cnt, P->sk_info,
                                     t16, t32, P->st));
    }
    int32_t cnt[4];
    int64_t r01[2];
    HIPCHK(hipMemcpyAsync(cnt, P->sk_cnt, sizeof(cnt), hipMemcpyDeviceToHost, P->st));
    HIPCHK(hipMemcpyAsync(&r01[0], w.row + n0, sizeof(int64_t), hipMemcpyDeviceToHost, P->st));
    HIPCHK(hipMemcpyAsync(&r01[1], w.row + n1, sizeof(int64_t), hipMemcpyDeviceToHost, P->st));
    HIPCHK(hipStreamSynchronize(P->st));
    const int64_t listed = (int64_t)cnt[0] + cnt[1] + cnt[2];
    const int64_t hcnt = r01[1] - r01[0];
    if (hcnt > P->sk_struts_cap) {
        if (P->sk_struts) HIPCHK(hipFree(P->sk_struts));
        P->sk_struts = nullptr;
        HIPCHK(hipMalloc((void **)&P->sk_struts, sizeof(int32_t) * (hcnt + 1)));
        P->sk_struts_cap = hcnt;
    }
    // record space for the listed nodes (first guess, then what they used)
    const double avg_deg = N > 0 ? 2.0 * (double)S / (double)N : 0.0;
    const int64_t per_node =
        lm::kRecHead + 4 + (int64_t)(avg_deg * (8 + 3 * lm::kRecArcFields + 3 + 2 * (k_avg + 4)) + 1);
    if ((rc = ensure_rec(P, listed * per_node + listed * per_node / 8 + 4096))) return rc;
    lm::Work wc = w;
    wc.queue = P->sk_lists;
    wc.cls_info = P->sk_info;
    for (int attempt = 0; attempt < 2; ++attempt) {
        HIPCHK(hipMemsetAsync(w.flags, 0, sizeof(int32_t), P->st));
        HIPCHK(hipMemsetAsync(w.flags + 2, 0, sizeof(int32_t), P->st));
        HIPCHK(hipMemsetAsync(w.rec_top, 0, sizeof(unsigned long long) * lm::kRecRegions, P->st));
        HIPCHK(hipMemsetAsync(w.work_ctr, 0, sizeof(int32_t) * 4, P->st));
        wc.rec = w.rec;
        wc.rec_words = w.rec_words;
        {
            PhaseTimer t(P, PH_NODE32);
            HIPCHK(lm::launch_node(P->in, wc, k, P->kappa_max, 0, P->st));
        }
        {
            PhaseTimer t(P, PH_NODE64);
            HIPCHK(lm::launch_node(P->in, wc, k, P->kappa_max, 1, P->st));
        }
        int32_t fl = 0;
        unsigned long long top[lm::kRecRegions];
        HIPCHK(hipMemcpyAsync(&fl, w.flags, sizeof(int32_t), hipMemcpyDeviceToHost, P->st));
        HIPCHK(hipMemcpyAsync(top, w.rec_top, sizeof(top), hipMemcpyDeviceToHost, P->st));
        HIPCHK(hipStreamSynchronize(P->st));
        if (!(fl & lm::DF_RECCAP)) break;
        if (attempt == 1) return LM_ERR_INTERNAL;
        unsigned long long mx = 0;
        for (int g = 0; g < lm::kRecRegions; ++g) mx = top[g] > mx ? top[g] : mx;
        if ((rc = ensure_rec(P, (int64_t)mx * lm::kRecRegions + (int64_t)mx))) return rc;
    }
    HIPCHK(hipMemsetAsync(P->sk_cnt + 4, 0, sizeof(int32_t), P->st));
    {
        PhaseTimer t(P, PH_EXPAND);
        HIPCHK(lm::launch_sink(P->in, w, n0, n1, hcnt, k, P->sk_struts, P->sk_cnt + 4, P->sk_slots, out_chunk,
                               node_part, out_parts, part_base, P->st));
    }
    return LM_OK;
}

}  // namespace

int lm_forward_sink(lm_plan *P, int k, int64_t chunk_nodes, uint64_t *d_out, int64_t n_chunks_cap)
{
    if (!P || !d_out || k < 3 || k > 4096 || chunk_nodes < 1) return LM_ERR_INVALID_ARG;
    const int64_t N = P->in.n_nodes;
    const int64_t nch = (N + chunk_nodes - 1) / chunk_nodes;
    if (nch > n_chunks_cap) return LM_ERR_CAPACITY;
    int rc = sink_alloc(P);
    if (rc) return rc;
    P->w.node_k = nullptr;
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t n0 = c * chunk_nodes, n1 = n0 + chunk_nodes < N ? n0 + chunk_nodes : N;
        if ((rc = sink_range(P, k, k, n0, n1, 4, 8, d_out + c * LM_SINK_WORDS, nullptr, nullptr, nullptr)))
            return rc;
    }
    // the node records now hold chunks: lm_fill / lm_backward need a new count
    P->k = 0;
    return LM_OK;
}

int lm_batched(lm_plan *P, int64_t n_parts, const int64_t *part_off, const int32_t *part_k, const lm_tuning *tune,
               uint64_t *d_out)
{
    if (!P || n_parts < 1 || !part_off || !part_k || !d_out) return LM_ERR_INVALID_ARG;
    const int64_t N = P->in.n_nodes;
    if (part_off[0] != 0 || part_off[n_parts] != N) return LM_ERR_INVALID_ARG;
    for (int64_t p = 0; p < n_parts; ++p)
        if (part_off[p + 1] < part_off[p] || part_k[p] < 3 || part_k[p] > 4096) return LM_ERR_INVALID_ARG;
    int t16 = 4, t32 = 8;
    int64_t group = (int64_t)1 << 23;
    if (tune) {
        if (tune->v_four_per_wave < 0 || tune->v_four_per_wave > 4 || tune->v_two_per_wave < tune->v_four_per_wave ||
            tune->v_two_per_wave > 8)
            return LM_ERR_INVALID_ARG;
        t16 = tune->v_four_per_wave;
        t32 = tune->v_two_per_wave;
        if (tune->group_nodes > 0) group = tune->group_nodes;
    }
    int rc = sink_alloc(P);
    if (rc) return rc;
    // per-node resolution and part, on the device
    int16_t *d_nk = nullptr;
    int32_t *d_np = nullptr, *d_pk = nullptr;
    int64_t *d_pb = nullptr;
    uint64_t *d_slots = nullptr;  // [n_parts][sink_slots_words()]
    const int64_t slot_words = n_parts * lm::sink_slots_words();
    if (hipMalloc((void **)&d_nk, sizeof(int16_t) * (N + 1)) != hipSuccess ||
        hipMalloc((void **)&d_np, sizeof(int32_t) * (N + 1)) != hipSuccess ||
        hipMalloc((void **)&d_pk, sizeof(int32_t) * (n_parts + 1)) != hipSuccess ||
        hipMalloc((void **)&d_pb, sizeof(int64_t) * (n_parts + 1)) != hipSuccess ||
        hipMalloc((void **)&d_slots, sizeof(uint64_t) * slot_words) != hipSuccess) {
        for (void *p : {(void *)d_nk, (void *)d_np, (void *)d_pk, (void *)d_pb, (void *)d_slots})
            if (p) (void)hipFree(p);
        return LM_ERR_HIP;
    }
    rc = LM_OK;
    if (hipMemcpyAsync(d_pb, part_off, sizeof(int64_t) * (n_parts + 1), hipMemcpyHostToDevice, P->st) !=
            hipSuccess ||
        hipMemcpyAsync(d_pk, part_k, sizeof(int32_t) * n_parts, hipMemcpyHostToDevice, P->st) != hipSuccess ||
        lm::launch_part_map(N, d_pb, d_pk, n_parts, d_np, d_nk, P->st) != hipSuccess ||
        hipMemsetAsync(d_slots, 0, sizeof(uint64_t) * slot_words, P->st) != hipSuccess)
        rc = LM_ERR_HIP;
    P->w.node_k = d_nk;
    // groups of whole parts of about `group` nodes: one node pass each
    for (int64_t p0 = 0; p0 < n_parts && rc == LM_OK;) {
        int64_t p1 = p0 + 1;
        while (p1 < n_parts && part_off[p1 + 1] - part_off[p0] <= group) ++p1;
        int kg = 3;
        for (int64_t p = p0; p < p1; ++p) kg = part_k[p] > kg ? part_k[p] : kg;
        rc = sink_range(P, kg, kg, part_off[p0], part_off[p1], t16, t32, nullptr, d_np, d_slots, d_pb);
        p0 = p1;
    }
    if (rc == LM_OK && lm::launch_parts_reduce((const unsigned long long *)d_slots, n_parts, d_out, P->st) !=
                           hipSuccess)
        rc = LM_ERR_HIP;
    (void)hipStreamSynchronize(P->st);
    P->w.node_k = nullptr;
    (void)hipFree(d_nk);
    (void)hipFree(d_np);
    (void)hipFree(d_pb);
    (void)hipFree(d_pk);
    (void)hipFree(d_slots);
    P->k = 0;
    return rc;
}

int lm_retriangulate(lm_plan *P, int k, const lm_outputs *out)
{
    if (!P || !out || !out->d_mesh_xyz || !out->d_tri || k < 3 || k > 4096) return LM_ERR_INVALID_ARG;
    if (P->k == 0) return LM_ERR_STATE;  // no meta-mesh from lm_count / lm_forward
    const int64_t N = P->in.n_nodes;
    if (!P->alt_index_mem) {
        const size_t top = sizeof(unsigned long long) * lm::kRecRegions, idx = sizeof(int64_t) * (N + 1);
        const size_t bytes = top + idx + sizeof(int32_t) * 8 + sizeof(int32_t) * (N + 1);
        HIPCHK(hipMalloc(&P->alt_index_mem, bytes));
        char *m = (char *)P->alt_index_mem;
        P->alt_rec_top = (unsigned long long *)m;
        P->alt_node_rec = (int64_t *)(m + top);
        P->redo_cnt = (int32_t *)(m + top + idx);
        P->redo = P->redo_cnt + 8;
    }
    // the slot that does not hold the meta-mesh receives the new records
    const bool base_in_w = P->base_slot == 0;
    const uint32_t *src_rec = base_in_w ? P->w.rec : P->alt_rec;
    const int64_t *src_node_rec = base_in_w ? P->w.node_rec : P->alt_node_rec;
    // records differ from the source's only in their loop samples, whose
    // count grows at most like k: scale the source slot's size
    const int64_t src_words = base_in_w ? P->w.rec_words : P->alt_rec_words;
    int64_t need = rec_estimate(P, k);
    if (k > P->k) {
        const int64_t scaled = (int64_t)((double)src_words * k / P->k);
        need = scaled > need ? scaled : need;
    } else if (src_words > need) {
        need = src_words;
    }
    const int64_t unit = 4 * lm::kRecRegions;
    need = (need + unit - 1) / unit * unit;
    lm::Work wd = P->w;
    if (base_in_w) {
        if (need > P->alt_rec_words) {
            HIPCHK(hipStreamSynchronize(P->st));
            if (P->alt_rec) HIPCHK(hipFree(P->alt_rec));
            P->alt_rec = nullptr;
            HIPCHK(hipMalloc((void **)&P->alt_rec, sizeof(uint32_t) * need));
            P->alt_rec_words = need;
        }
        wd.rec = P->alt_rec;
        wd.rec_words = P->alt_rec_words;
        wd.node_rec = P->alt_node_rec;
        wd.rec_top = P->alt_rec_top;
    } else if ((P->w.rec_words < need)) {
        int rc = ensure_rec(P, need);  // the current slot holds an earlier re-subdivision only
        if (rc) return rc;
        wd = P->w;
    }
    lm::FillOut f = to_fill(out);
    int rc = run_count(P, k, &f, wd, src_rec, src_node_rec, P->redo, P->redo_cnt);
    if (rc) return rc;
    rc = fill_common(P, k, f, out, wd);
    if (rc) return rc;
    if (base_in_w) {  // the new records become current; the meta-mesh moves to the other slot
        std::swap(P->w.rec, P->alt_rec);
        std::swap(P->w.rec_words, P->alt_rec_words);
        std::swap(P->w.node_rec, P->alt_node_rec);
        std::swap(P->w.rec_top, P->alt_rec_top);
        P->base_slot = 1;
    }
    P->last_on_host = false;
    return LM_OK;
}

int lm_arc_encode(lm_plan *P, const float *d_arc_f32, const uint32_t *d_arc_u32, int64_t n_arcs, int64_t ld,
                  float r_min, float r_max, const lm_arc_codes *c, int64_t *n_fallback)
{
    if (!P || !c || !n_fallback || n_arcs < 0 || ld < n_arcs || !(r_min > 0.f) || !(r_max >= r_min))
        return LM_ERR_INVALID_ARG;
    if (n_arcs > 0 && (!d_arc_f32 || !d_arc_u32 || !c->d_codes || !c->d_fallback_mask)) return LM_ERR_INVALID_ARG;
    if (c->cap_arcs < n_arcs || c->cap_fallback < 0 || (c->cap_fallback > 0 && !c->d_fallback))
        return LM_ERR_CAPACITY;
    *n_fallback = 0;
    if (n_arcs == 0) return LM_OK;
    if (!P->codec_ctr) HIPCHK(hipMalloc((void **)&P->codec_ctr, sizeof(unsigned long long)));
    HIPCHK(hipMemsetAsync(P->codec_ctr, 0, sizeof(unsigned long long), P->st));
    HIPCHK(hipMemsetAsync(c->d_fallback_mask, 0, sizeof(uint32_t) * ((n_arcs + 31) / 32), P->st));
    HIPCHK(lm::launch_arc_codec(P->in, P->w, true, d_arc_f32, d_arc_u32, n_arcs, ld, (double)r_min, (double)r_max,
                                c->d_codes, c->d_fallback_mask, c->d_fallback, c->cap_fallback, P->codec_ctr,
                                nullptr, 0, P->st));
    unsigned long long nf = 0;
    HIPCHK(hipMemcpyAsync(&nf, P->codec_ctr, sizeof(nf), hipMemcpyDeviceToHost, P->st));
    HIPCHK(hipStreamSynchronize(P->st));
    *n_fallback = (int64_t)nf;
    return (int64_t)nf > c->cap_fallback ? LM_ERR_CAPACITY : LM_OK;
}

int lm_arc_decode(lm_plan *P, const lm_arc_codes *c, const uint32_t *d_arc_u32, int64_t n_arcs, int64_t ld,
                  float r_min, float r_max, float *d_arc_f32_out, int64_t ld_out)
{
    if (!P || !c || n_arcs < 0 || ld < n_arcs || ld_out < n_arcs || !(r_min > 0.f) || !(r_max >= r_min))
        return LM_ERR_INVALID_ARG;
    if (n_arcs == 0) return LM_OK;
    if (!d_arc_u32 || !d_arc_f32_out || !c->d_codes || !c->d_fallback_mask) return LM_ERR_INVALID_ARG;
    if (c->cap_arcs < n_arcs) return LM_ERR_CAPACITY;
    HIPCHK(lm::launch_arc_codec(P->in, P->w, false, nullptr, d_arc_u32, n_arcs, ld, (double)r_min, (double)r_max,
                                c->d_codes, c->d_fallback_mask, c->d_fallback, c->cap_fallback, nullptr,
                                d_arc_f32_out, ld_out, P->st));
    return LM_OK;
}

int lm_read_totals(lm_plan *P, lm_totals *totals)
{
    if (!P || !totals) return LM_ERR_INVALID_ARG;
    int32_t fl;
    int rc = read_totals(P, totals, &fl);
    if (rc) return rc;
    if (fl & (lm::DF_CAPACITY | lm::DF_RECCAP)) return LM_ERR_CAPACITY;
    return LM_OK;
}

int lm_prepare(lm_plan *P)
{
    if (!P) return LM_ERR_INVALID_ARG;
    PhaseTimer t(P, PH_PREPARE);
    HIPCHK(hipMemsetAsync(P->w.flags + 1, 0, sizeof(int32_t), P->st));
    HIPCHK(lm::launch_prepare(P->in, P->w, P->st));
    return LM_OK;
}

int lm_set_profiling(lm_plan *P, int on)
{
    if (!P) return LM_ERR_INVALID_ARG;
    P->profiling = on != 0;
    return LM_OK;
}

int lm_get_profile(lm_plan *P, double *ms, int64_t *calls, int n)
{
    if (!P || !ms || !calls || n < PH_N) return LM_ERR_INVALID_ARG;
    for (int i = 0; i < PH_N; ++i) {
        ms[i] = 0.0;
        calls[i] = 0;
    }
    HIPCHK(hipStreamSynchronize(P->st));
    for (auto &e : P->ev) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, e.second.first, e.second.second));
        ms[e.first] += t;
        calls[e.first] += 1;
        P->pool.push_back(e.second.first);
        P->pool.push_back(e.second.second);
    }
    P->ev.clear();
    return LM_OK;
}

int lm_set_schedule(lm_plan *P, int schedule)
{
    if (!P || (schedule != LM_SCHEDULE_WAVE && schedule != LM_SCHEDULE_THREAD)) return LM_ERR_INVALID_ARG;
    P->schedule = schedule;
    return LM_OK;
}

int lm_set_precision(lm_plan *P, float kappa_max)
{
    if (!P || !(kappa_max >= 0.0f)) return LM_ERR_INVALID_ARG;
    P->kappa_max = kappa_max;
    P->k = 0;  // counts must be redone
    return LM_OK;
}

void lm_plan_destroy(lm_plan *P)
{
    if (!P) return;
    (void)hipStreamSynchronize(P->st);
    for (auto &e : P->ev) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    for (auto e : P->pool) (void)hipEventDestroy(e);
    if (P->w.rec) (void)hipFree(P->w.rec);
    for (void *p : {(void *)P->sk_mark, (void *)P->sk_lists, (void *)P->sk_cnt, (void *)P->sk_info,
                    (void *)P->sk_struts, (void *)P->sk_slots, (void *)P->alt_rec, P->alt_index_mem, (void *)P->codec_ctr, P->thread_scratch, P->grad_mem})
        if (p) (void)hipFree(p);
    (void)hipFree(P->ws);
    delete P;
}

const char *lm_status_string(int code)
{
    switch (code) {
    case LM_OK: return "ok";
    case LM_ERR_INVALID_ARG: return "invalid argument";
    case LM_ERR_BAD_LATTICE: return "strut endpoint out of range";
    case LM_ERR_CAPACITY: return "output buffer too small";
    case LM_ERR_UNSUPPORTED: return "size not supported by this library";
    case LM_ERR_HIP: return "HIP runtime error";
    case LM_ERR_STATE: return "call out of order";
    case LM_ERR_INTERNAL: return "workspace could not be sized";
    case LM_ERR_IO: return "file could not be written";
    default: return "unknown status";
    }
}

}  // extern "C"
