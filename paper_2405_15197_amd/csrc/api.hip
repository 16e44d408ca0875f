// Host side of the C ABI declared in include/latmesh.h.
#include <mutex>
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
    // device memory: library-owned (allocated here, at creation or at the
    // first use of a part) or all carved from the caller's workspace
    bool caller_ws = false;
    int32_t ws_flags = 0;       // LM_WS_* parts carved (caller workspace)
    void *ws = nullptr;         // fixed workspace (library-owned plans)
    // sink mode (LM_WS_SINK)
    void *sink_mem = nullptr;
    int32_t *sk_mark = nullptr;     // [N] epoch of the last range listing the node
    int32_t *sk_lists = nullptr;    // [kClasses][N + 1] range node lists
    int32_t *sk_cnt = nullptr;      // [8] list sizes, then the strut count
    int64_t *sk_info = nullptr;     // [8] class sizes / starts for the node kernel
    int32_t *sk_struts = nullptr;   // [S + 1] struts owned by the range
    int32_t *sk_fail = nullptr;     // [N + 1] per range: records overflowed
    unsigned long long *sk_slots = nullptr;  // chunk-mode slots
    int32_t sk_epoch = 0;
    // batched parts (with the sink part)
    void *batch_mem = nullptr, *batch_parts_mem = nullptr;
    int16_t *bt_node_k = nullptr;   // [N + 1] resolution of each node
    int32_t *bt_node_part = nullptr;// [N + 1] part of each node
    int64_t *bt_part_base = nullptr;// [cap + 1] first node of each part
    int32_t *bt_part_k = nullptr;   // [cap + 1]
    unsigned long long *bt_slots = nullptr;  // [cap][sink_slots_words]
    int64_t bt_cap = 0;
    // second record slot (re-subdivision): records, node record index, bump
    // counters; base_slot says where the meta-mesh of the last count is
    uint32_t *alt_rec = nullptr;
    int64_t alt_rec_words = 0;
    int64_t *alt_node_rec = nullptr;
    unsigned long long *alt_rec_top = nullptr;
    int base_slot = 0;
    // the allocation behind the second node record index and counters (the
    // pointers above swap with the workspace's own at every switch), and the
    // redo lists [N] and their counters [8]
    void *alt_index_mem = nullptr;
    int32_t *redo = nullptr;
    int32_t *redo_cnt = nullptr;
    unsigned long long *codec_ctr = nullptr;  // fallback counter of lm_arc_encode
    void *grad_mem = nullptr;                 // adjoint scratch (library-owned)
    int schedule = LM_SCHEDULE_WAVE;          // FP32 node pass of lm_count / lm_forward
    void *thread_scratch = nullptr;           // per-node scratch of the thread-centric pass
    int64_t cls_est[4];        // nodes per valence class when the plan was made (grid sizes only)
    bool has_cls_est = false;
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

// Hands out 256-byte aligned pieces of one buffer; with base == nullptr it
// only adds up the sizes.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <typename T>
    T *take(int64_t count)
    {
        char *p = base ? base + off : nullptr;
        off += align_up(sizeof(T) * (size_t)(count > 0 ? count : 0));
        return (T *)p;
    }
};

// The fixed workspace: adjacency, counts, offsets, queues, flags.
void carve_fixed(lm_plan *P, Carver &c, int64_t N, int64_t S)
{
    lm::Work &w = P->w;
    const int64_t H = 2 * S;
    w.node4 = c.take<float4>(N + 1);
    w.row = c.take<int64_t>(N + 1);
    w.he = c.take<int2>(H + 1);
    w.deg = c.take<int32_t>(N + 1);
    w.strut_he = c.take<int64_t>(H + 1);
    w.node_cnt = c.take<int32_t>((int64_t)lm::kNodeCols * (N + 1));
    w.node_off = c.take<int64_t>((int64_t)lm::kNodeScanCols * (N + 1));
    w.he_len = c.take<int32_t>(H + 1);
    w.he_loop = c.take<int64_t>(H + 1);
    w.he_rot = c.take<int32_t>(H + 1);
    w.band_cnt = c.take<int32_t>(S + 1);
    w.band_off = c.take<int64_t>(S + 1);
    int64_t tl = lm::scan_tmp_needed(N, lm::kNodeScanCols);
    const int64_t t2 = lm::scan_tmp_needed(S, 1);
    if (t2 > tl) tl = t2;
    w.scan_tmp = c.take<int64_t>(tl);
    w.scan_tmp_len = tl;
    w.flags = c.take<int32_t>(4);
    w.totals = c.take<int64_t>(16);
    w.fb_list = c.take<int32_t>(N + 1);
    w.node_rec = c.take<int64_t>(N + 1);
    w.rec_top = c.take<unsigned long long>(lm::kRecRegions);
    w.queue = c.take<int32_t>(N + 1);
    w.cls_info = c.take<int64_t>(8);
    w.work_ctr = c.take<int32_t>(8);
    P->codec_ctr = c.take<unsigned long long>(1);
    w.node_k = nullptr;
}

void carve_grad(lm_plan *P, Carver &c, int64_t N, int64_t S)
{
    P->w.loss_node = c.take<double>(3 * (N + 1) + 3 * 256);  // node terms, then block partials
    P->w.grad_node = c.take<float>(4 * (N + 1));
    P->w.grad_he = c.take<float>(4 * (2 * S + 1));
}

void carve_sink(lm_plan *P, Carver &c, int64_t N, int64_t S)
{
    P->sk_mark = c.take<int32_t>(N + 1);
    P->sk_lists = c.take<int32_t>((int64_t)lm::kClasses * (N + 1));
    P->sk_cnt = c.take<int32_t>(8);
    P->sk_info = c.take<int64_t>(8);
    P->sk_struts = c.take<int32_t>(S + 1);
    P->sk_fail = c.take<int32_t>(N + 1);
    P->sk_slots = c.take<unsigned long long>(lm::sink_slots_words());
}

void carve_batch_nodes(lm_plan *P, Carver &c, int64_t N)
{
    P->bt_node_k = c.take<int16_t>(N + 1);
    P->bt_node_part = c.take<int32_t>(N + 1);
}

void carve_batch_parts(lm_plan *P, Carver &c, int64_t cap)
{
    P->bt_part_base = c.take<int64_t>(cap + 1);
    P->bt_part_k = c.take<int32_t>(cap + 1);
    P->bt_slots = c.take<unsigned long long>(cap * lm::sink_slots_words());
    P->bt_cap = cap;
}

void carve_retri_index(lm_plan *P, Carver &c, int64_t N)
{
    P->alt_rec_top = c.take<unsigned long long>(lm::kRecRegions);
    P->alt_node_rec = c.take<int64_t>(N + 1);
    P->redo_cnt = c.take<int32_t>(8);
    P->redo = c.take<int32_t>(N + 1);
}

// Node-record words of the whole lattice at resolution k: per node the
// header and about 2 vertices, 3 arcs and a hole per incident strut; per
// half-edge a loop of about k samples and about k / 2 interior points.
int64_t rec_estimate_nk(int64_t N, int64_t S, int k)
{
    const int64_t H = 2 * S;
    int64_t words = N * (lm::kRecHead + 4) +
                    H * (2 * 4 + 3 * lm::kRecArcFields + 3 + 2 * (int64_t)(k + 4) + 3 * (int64_t)(k / 2 + 2));
    return words + words / 8 + 4096;
}
int64_t rec_estimate(const lm_plan *P, int k) { return rec_estimate_nk(P->in.n_nodes, P->in.n_struts, k); }

inline int64_t rec_round(int64_t words)
{
    const int64_t unit = 4 * lm::kRecRegions;
    return (words + unit - 1) / unit * unit;
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

// Node pass (meta-meshing at k, or with src_rec set the re-subdivision of
// the meta-mesh in those records) into the records of w, then band counts,
// prefix sums and device totals (and capacity flags when out != nullptr).
int run_count(lm_plan *P, int k, const lm::FillOut *out, const lm::Work &w, const uint32_t *src_rec = nullptr,
              const int64_t *src_node_rec = nullptr, int32_t *redo = nullptr, int32_t *redo_cnt = nullptr)
{
    const int64_t N = P->in.n_nodes, S = P->in.n_struts;
    // flags[0] (count / fill) and flags[2] (FP64 hand-over count)
    HIPCHK(hipMemsetAsync(w.flags, 0, sizeof(int32_t), P->st));
    HIPCHK(hipMemsetAsync(w.flags + 2, 0, sizeof(int32_t), P->st));
    HIPCHK(hipMemsetAsync(w.totals, 0, sizeof(int64_t) * 16, P->st));
    HIPCHK(hipMemsetAsync(w.rec_top, 0, sizeof(unsigned long long) * lm::kRecRegions, P->st));
    HIPCHK(hipMemsetAsync(w.work_ctr, 0, sizeof(int32_t) * 8, P->st));
    {
        PhaseTimer t(P, PH_NODE32);
        if (redo_cnt) HIPCHK(hipMemsetAsync(redo_cnt, 0, sizeof(int32_t) * 8, P->st));
        if (P->schedule == LM_SCHEDULE_THREAD && !src_rec) {
            if (!P->thread_scratch) HIPCHK(hipMalloc(&P->thread_scratch, lm::node_thread_scratch_bytes()));
            HIPCHK(lm::launch_node_thread(P->in, w, k, P->kappa_max, P->thread_scratch, P->st));
        } else {
            HIPCHK(lm::launch_node(P->in, w, k, P->kappa_max, 0, P->st, src_rec, src_node_rec, redo, redo_cnt,
                                   nullptr, P->has_cls_est ? P->cls_est : nullptr));
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
// A caller-owned workspace has a fixed record space: LM_ERR_CAPACITY when
// it is smaller.
int ensure_rec(lm_plan *P, int64_t words)
{
    words = rec_round(words);
    if (words <= P->w.rec_words) return LM_OK;
    if (P->caller_ws) return LM_ERR_CAPACITY;
    HIPCHK(hipStreamSynchronize(P->st));
    if (P->w.rec) HIPCHK(hipFree(P->w.rec));
    P->w.rec = nullptr;
    P->w.rec_words = 0;
    HIPCHK(hipMalloc((void **)&P->w.rec, sizeof(uint32_t) * words));
    P->w.rec_words = words;
    return LM_OK;
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

int check_lattice(const lm_lattice *lat, bool need_radius = true)
{
    if (!lat || lat->n_nodes < 0 || lat->n_struts < 0) return LM_ERR_INVALID_ARG;
    if (lat->n_nodes > 0 && (!lat->d_x || !lat->d_y || !lat->d_z || (need_radius && !lat->d_radius)))
        return LM_ERR_INVALID_ARG;
    if (lat->n_struts > 0 && (!lat->d_strut_a || !lat->d_strut_b)) return LM_ERR_INVALID_ARG;
    // node and strut ids are int32; half-edge indices are int64
    if (lat->n_nodes >= ((int64_t)1 << 31) || lat->n_struts >= ((int64_t)1 << 31)) return LM_ERR_UNSUPPORTED;
    return LM_OK;
}

void init_plan(lm_plan *P, const lm_lattice *lat, void *stream)
{
    P->st = (hipStream_t)stream;
    P->in.n_nodes = lat->n_nodes;
    P->in.n_struts = lat->n_struts;
    P->in.x = lat->d_x;
    P->in.y = lat->d_y;
    P->in.z = lat->d_z;
    P->in.r = lat->d_radius;
    P->in.sa = lat->d_strut_a;
    P->in.sb = lat->d_strut_b;
    P->w.rec = nullptr;
    P->w.rec_words = 0;
    P->w.loss_node = nullptr;
    P->w.grad_node = nullptr;
    P->w.grad_he = nullptr;
    P->k = 0;
    P->kappa_max = 32.0f;
    P->profiling = false;
}

lm_plan *new_plan(const lm_lattice *lat, void *stream)
{
    lm_plan *P = new (std::nothrow) lm_plan();
    if (!P) return nullptr;
    init_plan(P, lat, stream);
    return P;
}

// Validation and adjacency of a new plan (synchronises).
int first_prepare(lm_plan *P)
{
    int32_t fl = 0;
    if (hipMemsetAsync(P->w.flags, 0, sizeof(int32_t) * 4, P->st) != hipSuccess ||
        hipMemsetAsync(P->w.totals, 0, sizeof(int64_t) * 16, P->st) != hipSuccess ||
        lm::launch_prepare(P->in, P->w, P->st) != hipSuccess ||
        hipMemcpyAsync(&fl, P->w.flags + 1, sizeof(int32_t), hipMemcpyDeviceToHost, P->st) != hipSuccess ||
        hipMemcpyAsync(P->cls_est, P->w.cls_info, sizeof(P->cls_est), hipMemcpyDeviceToHost, P->st) != hipSuccess ||
        hipStreamSynchronize(P->st) != hipSuccess)
        return LM_ERR_HIP;
    if (fl & lm::DF_BADLAT) return LM_ERR_BAD_LATTICE;  // set in flags[1]
    P->has_cls_est = true;
    return LM_OK;
}

// Carves (or, with base null, sizes) every part of a caller-owned workspace.
size_t ws_layout(lm_plan *P, void *base, int64_t N, int64_t S, const lm_options &o)
{
    Carver c(base);
    carve_fixed(P, c, N, S);
    if (o.flags & LM_WS_GRADIENT) carve_grad(P, c, N, S);
    if (o.flags & LM_WS_SINK) {
        carve_sink(P, c, N, S);
        carve_batch_nodes(P, c, N);
        carve_batch_parts(P, c, o.max_parts);
    }
    const int64_t rw = rec_round(o.record_bytes > 0 ? (o.record_bytes + 3) / 4 : rec_estimate_nk(N, S, o.k_max));
    if (o.flags & LM_WS_RETRI) {
        carve_retri_index(P, c, N);
        P->alt_rec = c.take<uint32_t>(rw);
        P->alt_rec_words = rw;
    }
    P->w.rec = c.take<uint32_t>(rw);
    P->w.rec_words = rw;
    return c.off;
}

int check_options(const lm_options *opt, lm_options *o)
{
    lm_options d;
    d.flags = 0;
    d.k_max = 16;
    d.record_bytes = 0;
    d.max_parts = 0;
    *o = opt ? *opt : d;
    if (o->k_max < 3 || o->k_max > 4096 || o->record_bytes < 0 || o->max_parts < 0 ||
        (o->flags & ~(LM_WS_SINK | LM_WS_GRADIENT | LM_WS_RETRI)))
        return LM_ERR_INVALID_ARG;
    return LM_OK;
}

}  // namespace

extern "C" {

int lm_workspace_size(int64_t n_nodes, int64_t n_struts, const lm_options *opt, size_t *bytes)
{
    if (!bytes || n_nodes < 0 || n_struts < 0) return LM_ERR_INVALID_ARG;
    if (n_nodes >= ((int64_t)1 << 31) || n_struts >= ((int64_t)1 << 31)) return LM_ERR_UNSUPPORTED;
    lm_options o;
    int rc = check_options(opt, &o);
    if (rc) return rc;
    lm_plan tmp;
    *bytes = ws_layout(&tmp, nullptr, n_nodes, n_struts, o);
    return LM_OK;
}

int lm_plan_create_in(lm_plan **plan, const lm_lattice *lat, const lm_options *opt, void *d_workspace,
                      size_t workspace_bytes, void *stream)
{
    if (!plan) return LM_ERR_INVALID_ARG;
    *plan = nullptr;
    int rc = check_lattice(lat);
    if (rc) return rc;
    lm_options o;
    if ((rc = check_options(opt, &o))) return rc;
    if (!d_workspace || ((uintptr_t)d_workspace & 255)) return LM_ERR_INVALID_ARG;
    lm_plan *P = new_plan(lat, stream);
    if (!P) return LM_ERR_INTERNAL;
    P->caller_ws = true;
    P->ws_flags = o.flags;
    if (ws_layout(P, nullptr, lat->n_nodes, lat->n_struts, o) > workspace_bytes) {
        delete P;
        return LM_ERR_CAPACITY;
    }
    ws_layout(P, d_workspace, lat->n_nodes, lat->n_struts, o);
    if (o.flags & LM_WS_SINK) {
        if (hipMemsetAsync(P->sk_mark, 0, sizeof(int32_t) * (lat->n_nodes + 1), P->st) != hipSuccess ||
            hipMemsetAsync(P->sk_slots, 0, sizeof(unsigned long long) * lm::sink_slots_words(), P->st) !=
                hipSuccess) {
            delete P;
            return LM_ERR_HIP;
        }
    }
    if ((rc = first_prepare(P))) {
        delete P;
        return rc;
    }
    *plan = P;
    return LM_OK;
}

int lm_plan_create(lm_plan **plan, const lm_lattice *lat, void *stream)
{
    if (!plan) return LM_ERR_INVALID_ARG;
    *plan = nullptr;
    int rc = check_lattice(lat);
    if (rc) return rc;
    lm_plan *P = new_plan(lat, stream);
    if (!P) return LM_ERR_INTERNAL;
    Carver c0(nullptr);
    carve_fixed(P, c0, lat->n_nodes, lat->n_struts);
    if (hipMalloc(&P->ws, c0.off) != hipSuccess) {
        delete P;
        return LM_ERR_HIP;
    }
    Carver c(P->ws);
    carve_fixed(P, c, lat->n_nodes, lat->n_struts);
    if ((rc = first_prepare(P))) {
        (void)hipFree(P->ws);
        delete P;
        return rc;
    }
    *plan = P;
    return LM_OK;
}

int lm_plan_create_end_radii(lm_plan **plan, const lm_lattice *lat, const float *d_end_radius, float rel_tol,
                             float *d_radius, int64_t *n_mismatch, void *stream)
{
    if (!plan) return LM_ERR_INVALID_ARG;
    *plan = nullptr;
    if (n_mismatch) *n_mismatch = 0;
    int rc = check_lattice(lat, false);
    if (rc) return rc;
    if (!(rel_tol >= 0.f) || (lat->n_struts > 0 && !d_end_radius) || (lat->n_nodes > 0 && !d_radius))
        return LM_ERR_INVALID_ARG;
    lm_lattice l2 = *lat;
    l2.d_radius = d_radius;  // read by the plan from here on
    lm_plan *P = nullptr;
    // the adjacency does not depend on the radii: build it, derive the radii,
    // then redo the preparation with them
    if ((rc = lm_plan_create(&P, &l2, stream))) return rc;
    int32_t mism = 0;
    if (hipMemsetAsync(P->w.flags + 3, 0, sizeof(int32_t), P->st) != hipSuccess ||
        lm::launch_end_radii(P->in, P->w, d_end_radius, rel_tol, d_radius, P->w.flags + 3, P->st) != hipSuccess ||
        hipMemcpyAsync(&mism, P->w.flags + 3, sizeof(int32_t), hipMemcpyDeviceToHost, P->st) != hipSuccess ||
        hipStreamSynchronize(P->st) != hipSuccess) {
        lm_plan_destroy(P);
        return LM_ERR_HIP;
    }
    if (n_mismatch) *n_mismatch = mism;
    if (mism) {
        lm_plan_destroy(P);
        return LM_ERR_RADIUS_MISMATCH;
    }
    if ((rc = first_prepare(P))) {
        lm_plan_destroy(P);
        return rc;
    }
    *plan = P;
    return LM_OK;
}

int lm_end_radius_gradient(lm_plan *P, const float *d_grad_radius, float *d_grad_end)
{
    if (!P || (P->in.n_struts > 0 && (!d_grad_radius || !d_grad_end))) return LM_ERR_INVALID_ARG;
    HIPCHK(lm::launch_end_grad(P->in, P->w, d_grad_radius, d_grad_end, P->st));
    return LM_OK;
}

int lm_count(lm_plan *P, int k, lm_totals *totals)
{
    if (!P || !totals || k < 3 || k > 4096) return LM_ERR_INVALID_ARG;
    int rc = LM_OK;
    if (P->w.rec_words == 0 && (rc = ensure_rec(P, rec_estimate(P, k)))) return rc;
    int32_t fl = 0;
    P->k = 0;
    P->last_on_host = false;
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

}  // extern "C"

namespace {

// Scratch of lm_loss and lm_backward: per-node loss terms, per-node and
// per-half-edge adjoint partials (library-owned: allocated at the first use).
int grad_alloc(lm_plan *P)
{
    if (P->w.grad_he) return LM_OK;
    if (P->caller_ws) return LM_ERR_UNSUPPORTED;
    Carver c0(nullptr);
    carve_grad(P, c0, P->in.n_nodes, P->in.n_struts);
    HIPCHK(hipMalloc(&P->grad_mem, c0.off));
    Carver c(P->grad_mem);
    carve_grad(P, c, P->in.n_nodes, P->in.n_struts);
    return LM_OK;
}

}  // namespace

extern "C" {

int lm_loss(lm_plan *P, const lm_outputs *out, const lm_loss_weights *w, double *d_terms, float *d_dl_dx)
{
    if (!P || !out || !w || !d_terms || !d_dl_dx || !out->d_mesh_xyz || !out->d_tri) return LM_ERR_INVALID_ARG;
    if (P->k == 0) return LM_ERR_STATE;
    if (out->cap_mesh_vertices < 0 || out->cap_triangles < 0) return LM_ERR_INVALID_ARG;
    // sizes known on the host (after lm_count): refuse small buffers before
    // any launch; otherwise the kernels check the device totals and skip
    // (lm_read_totals then reports LM_ERR_CAPACITY)
    if (P->last_on_host &&
        (out->cap_mesh_vertices < P->last.n_mesh_vertices || out->cap_triangles < P->last.n_triangles))
        return LM_ERR_CAPACITY;
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

}  // extern "C"

namespace {

// Sink-mode buffers (library-owned: allocated at the first use).
int sink_alloc(lm_plan *P)
{
    if (P->sk_mark) return LM_OK;
    if (P->caller_ws) return LM_ERR_UNSUPPORTED;
    const int64_t N = P->in.n_nodes, S = P->in.n_struts;
    Carver c0(nullptr);
    carve_sink(P, c0, N, S);
    HIPCHK(hipMalloc(&P->sink_mem, c0.off));
    Carver c(P->sink_mem);
    carve_sink(P, c, N, S);
    HIPCHK(hipMemsetAsync(P->sk_mark, 0, sizeof(int32_t) * (N + 1), P->st));
    HIPCHK(hipMemsetAsync(P->sk_slots, 0, sizeof(unsigned long long) * lm::sink_slots_words(), P->st));
    return LM_OK;
}

// Batched-part buffers for n_parts parts (library-owned: per-node arrays at
// the first use, per-part arrays grown when a call has more parts).
int batch_alloc(lm_plan *P, int64_t n_parts)
{
    if (P->caller_ws) return n_parts <= P->bt_cap ? LM_OK : LM_ERR_CAPACITY;
    if (!P->batch_mem) {
        Carver c0(nullptr);
        carve_batch_nodes(P, c0, P->in.n_nodes);
        HIPCHK(hipMalloc(&P->batch_mem, c0.off));
        Carver c(P->batch_mem);
        carve_batch_nodes(P, c, P->in.n_nodes);
    }
    if (n_parts > P->bt_cap) {
        HIPCHK(hipStreamSynchronize(P->st));
        if (P->batch_parts_mem) HIPCHK(hipFree(P->batch_parts_mem));
        P->batch_parts_mem = nullptr;
        P->bt_cap = 0;
        Carver c0(nullptr);
        carve_batch_parts(P, c0, n_parts);
        HIPCHK(hipMalloc(&P->batch_parts_mem, c0.off));
        Carver c(P->batch_parts_mem);
        carve_batch_parts(P, c, n_parts);
    }
    return LM_OK;
}

// One sink-mode range [n0, n1), queued without host synchronisation: its
// node list (range + higher-id halo) in valence classes (limits t16 / t32),
// the node pass in sink mode, the range's failure flag, then the bands.
// Chunk mode (out_chunk set): the range's words reduced into out_chunk.
int sink_range(lm_plan *P, int k, int64_t r, int64_t n0, int64_t n1, int t16, int t32, lm::SinkOut so,
               uint64_t *out_chunk)
{
    const int64_t N = P->in.n_nodes;
    lm::Work &w = P->w;
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
    lm::Work wc = w;
    wc.queue = P->sk_lists;
    wc.cls_info = P->sk_info;
    HIPCHK(hipMemsetAsync(w.rec_top, 0, sizeof(unsigned long long) * lm::kRecRegions, P->st));
    HIPCHK(hipMemsetAsync(w.work_ctr, 0, sizeof(int32_t) * 8, P->st));
    so.n0 = n0;
    so.n1 = n1;
    {
        PhaseTimer t(P, PH_NODE32);
        HIPCHK(lm::launch_node(P->in, wc, k, P->kappa_max, 0, P->st, nullptr, nullptr, nullptr, nullptr, &so));
    }
    {
        PhaseTimer t(P, PH_NODE64);
        HIPCHK(lm::launch_node(P->in, wc, k, P->kappa_max, 1, P->st, nullptr, nullptr, nullptr, nullptr, &so));
    }
    HIPCHK(lm::launch_range_done(w.flags, P->sk_fail, r, P->st));
    HIPCHK(hipMemsetAsync(P->sk_cnt + 4, 0, sizeof(int32_t), P->st));
    {
        PhaseTimer t(P, PH_ZIP);
        HIPCHK(lm::launch_sink_bands(P->in, w, n0, n1, k, P->sk_struts, P->sk_cnt + 4, so, P->st));
    }
    if (out_chunk) HIPCHK(lm::launch_sink_reduce(P->sk_slots, out_chunk, P->st));
    return LM_OK;
}

// Ranges bound[r] .. bound[r + 1] run back to back, then one
// synchronisation; a range whose records did not fit runs again after the
// record space grows (part mode: its parts' slots cleared first).
// rec_words: the record space the largest range is expected to need.
int sink_ranges(lm_plan *P, const std::vector<int64_t> &bound, const std::vector<int> &kmax, int t16, int t32,
                const lm::SinkOut &so, uint64_t *d_out_chunks, const std::vector<int64_t> *pbound,
                int64_t rec_words)
{
    const int64_t R = (int64_t)bound.size() - 1;
    int rc = ensure_rec(P, rec_words);
    if (rc && rc != LM_ERR_CAPACITY) return rc;  // caller-owned space: try with what there is
    HIPCHK(hipMemsetAsync(P->w.flags, 0, sizeof(int32_t) * 3, P->st));
    HIPCHK(hipMemsetAsync(P->sk_fail, 0, sizeof(int32_t) * (R + 1), P->st));
    for (int64_t r = 0; r < R; ++r)
        if ((rc = sink_range(P, kmax[r], r, bound[r], bound[r + 1], t16, t32, so,
                             d_out_chunks ? d_out_chunks + r * LM_SINK_WORDS : nullptr)))
            return rc;
    std::vector<int32_t> fail(R > 0 ? R : 1);
    if (R > 0) HIPCHK(hipMemcpyAsync(fail.data(), P->sk_fail, sizeof(int32_t) * R, hipMemcpyDeviceToHost, P->st));
    HIPCHK(hipStreamSynchronize(P->st));
    for (int64_t r = 0; r < R; ++r) {
        if (!fail[r]) continue;
        for (int attempt = 0; attempt < 2; ++attempt) {
            // the records of the range's nodes did not fit: grow by what the
            // fullest region needed, run the range again
            unsigned long long top[lm::kRecRegions];
            HIPCHK(hipMemcpyAsync(top, P->w.rec_top, sizeof(top), hipMemcpyDeviceToHost, P->st));
            HIPCHK(hipStreamSynchronize(P->st));
            unsigned long long mx = 0;
            for (int g = 0; g < lm::kRecRegions; ++g) mx = top[g] > mx ? top[g] : mx;
            if ((rc = ensure_rec(P, (int64_t)mx * lm::kRecRegions + P->w.rec_words / 4))) return rc;
            if (pbound) HIPCHK(lm::launch_clear_parts(so.out_parts, (*pbound)[r], (*pbound)[r + 1], P->st));
            HIPCHK(hipMemsetAsync(P->w.flags, 0, sizeof(int32_t) * 3, P->st));
            if ((rc = sink_range(P, kmax[r], r, bound[r], bound[r + 1], t16, t32, so,
                                 d_out_chunks ? d_out_chunks + r * LM_SINK_WORDS : nullptr)))
                return rc;
            int32_t f = 0;
            HIPCHK(hipMemcpyAsync(&f, P->sk_fail + r, sizeof(int32_t), hipMemcpyDeviceToHost, P->st));
            HIPCHK(hipStreamSynchronize(P->st));
            if (!f) break;
            if (attempt == 1) return LM_ERR_INTERNAL;
        }
    }
    return LM_OK;
}

// Record words of a sink range whose nodes, times their resolution plus 4,
// sum to nodes_k (the loops: per half-edge about k + 4 samples of two
// words), with a halo of `halo` times as many nodes again.
int64_t sink_rec_words(const lm_plan *P, double nodes_k, double halo)
{
    const int64_t N = P->in.n_nodes, S = P->in.n_struts;
    const double deg = N > 0 ? 2.0 * (double)S / (double)N : 0.0;
    return (int64_t)(deg * 2.0 * nodes_k * (1.0 + halo) * 1.15) + 4096;
}

}  // namespace

extern "C" {

int lm_forward_sink(lm_plan *P, int k, int64_t chunk_nodes, uint64_t *d_out, int64_t n_chunks_cap)
{
    if (!P || !d_out || k < 3 || k > 4096 || chunk_nodes < 1) return LM_ERR_INVALID_ARG;
    const int64_t N = P->in.n_nodes;
    const int64_t nch = (N + chunk_nodes - 1) / chunk_nodes;
    if (nch > n_chunks_cap) return LM_ERR_CAPACITY;
    int rc = sink_alloc(P);
    if (rc) return rc;
    P->w.node_k = nullptr;
    P->k = 0;  // the node records will hold chunks: lm_fill / lm_backward need a new count
    P->last_on_host = false;
    if (nch == 0) return LM_OK;
    std::vector<int64_t> bound(nch + 1);
    std::vector<int> kmax(nch, k);
    for (int64_t c = 0; c <= nch; ++c) bound[c] = c * chunk_nodes < N ? c * chunk_nodes : N;
    const int64_t largest = chunk_nodes < N ? chunk_nodes : N;
    lm::SinkOut so{0, 0, P->sk_slots, nullptr, nullptr, nullptr};
    return sink_ranges(P, bound, kmax, 4, 8, so, d_out, nullptr,
                       sink_rec_words(P, (double)largest * (k + 4), largest < N ? 0.5 : 0.0));
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
    int64_t group = 0;
    if (tune) {
        if (tune->v_four_per_wave < 0 || tune->v_four_per_wave > 4 || tune->v_two_per_wave < tune->v_four_per_wave ||
            tune->v_two_per_wave > 8 || tune->group_nodes < 0)
            return LM_ERR_INVALID_ARG;
        t16 = tune->v_four_per_wave;
        t32 = tune->v_two_per_wave;
        group = tune->group_nodes;
    }
    int rc = sink_alloc(P);
    if (rc) return rc;
    if ((rc = batch_alloc(P, n_parts))) return rc;
    P->k = 0;
    P->last_on_host = false;
    // groups of whole parts, each one node pass over all its parts' nodes.
    // Automatic: all parts at once when their records fit (a share of the
    // free device memory, or the caller's record space), else the fewest
    // groups that do.
    std::vector<double> nk(n_parts);  // nodes x (k + 4) per part
    for (int64_t p = 0; p < n_parts; ++p) nk[p] = (double)(part_off[p + 1] - part_off[p]) * (part_k[p] + 4);
    int64_t budget_words;
    if (P->caller_ws) {
        budget_words = P->w.rec_words;
    } else {
        size_t fr = 0, tot = 0;
        HIPCHK(hipMemGetInfo(&fr, &tot));
        budget_words = (int64_t)((double)(fr + sizeof(uint32_t) * (size_t)P->w.rec_words) * 0.7 / 4.0);
    }
    std::vector<int64_t> bound{0}, pbound{0};
    std::vector<int> kmax;
    double largest = 0.0;
    for (int64_t p0 = 0; p0 < n_parts;) {
        int64_t p1 = p0 + 1;
        double s = nk[p0];
        int kg = part_k[p0];
        while (p1 < n_parts) {
            const bool fits = group > 0 ? part_off[p1 + 1] - part_off[p0] <= group
                                        : sink_rec_words(P, s + nk[p1], 0.0) <= budget_words;
            if (!fits) break;
            s += nk[p1];
            kg = part_k[p1] > kg ? part_k[p1] : kg;
            ++p1;
        }
        largest = s > largest ? s : largest;
        bound.push_back(part_off[p1]);
        pbound.push_back(p1);
        kmax.push_back(kg);
        p0 = p1;
    }
    // per-node resolution and part, on the device
    HIPCHK(hipMemcpyAsync(P->bt_part_base, part_off, sizeof(int64_t) * (n_parts + 1), hipMemcpyHostToDevice, P->st));
    HIPCHK(hipMemcpyAsync(P->bt_part_k, part_k, sizeof(int32_t) * n_parts, hipMemcpyHostToDevice, P->st));
    HIPCHK(lm::launch_part_map(N, P->bt_part_base, P->bt_part_k, n_parts, P->bt_node_part, P->bt_node_k, P->st));
    HIPCHK(lm::launch_clear_parts(P->bt_slots, 0, n_parts, P->st));
    P->w.node_k = P->bt_node_k;
    lm::SinkOut so{0, 0, nullptr, P->bt_node_part, P->bt_slots, P->bt_part_base};
    rc = sink_ranges(P, bound, kmax, t16, t32, so, nullptr, &pbound, sink_rec_words(P, largest, 0.0));
    if (rc == LM_OK && lm::launch_parts_reduce(P->bt_slots, n_parts, d_out, P->st) != hipSuccess) rc = LM_ERR_HIP;
    if (rc == LM_OK && hipStreamSynchronize(P->st) != hipSuccess) rc = LM_ERR_HIP;
    P->w.node_k = nullptr;
    return rc;
}

int lm_retriangulate(lm_plan *P, int k, const lm_outputs *out)
{
    if (!P || !out || !out->d_mesh_xyz || !out->d_tri || k < 3 || k > 4096) return LM_ERR_INVALID_ARG;
    if (P->k == 0) return LM_ERR_STATE;  // no meta-mesh from lm_count / lm_forward
    if (P->caller_ws && !(P->ws_flags & LM_WS_RETRI)) return LM_ERR_UNSUPPORTED;
    const int64_t N = P->in.n_nodes;
    if (!P->alt_node_rec) {
        Carver c0(nullptr);
        carve_retri_index(P, c0, N);
        HIPCHK(hipMalloc(&P->alt_index_mem, c0.off));
        Carver c(P->alt_index_mem);
        carve_retri_index(P, c, N);
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
    need = rec_round(need);
    lm::Work wd = P->w;
    if (base_in_w) {
        if (need > P->alt_rec_words && !P->caller_ws) {
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
    } else if (P->w.rec_words < need && !P->caller_ws) {
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
    // the ablation's per-node scratch (gigabytes) is never carved from a caller's workspace
    if (P->caller_ws && schedule == LM_SCHEDULE_THREAD) return LM_ERR_UNSUPPORTED;
    P->schedule = schedule;
    return LM_OK;
}

int lm_set_precision(lm_plan *P, float kappa_max)
{
    if (!P || !(kappa_max >= 0.0f)) return LM_ERR_INVALID_ARG;
    P->kappa_max = kappa_max;
    P->k = 0;  // counts must be redone
    P->last_on_host = false;
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
    if (!P->caller_ws) {
        for (void *p : {(void *)P->w.rec, P->ws, P->sink_mem, P->batch_mem, P->batch_parts_mem, (void *)P->alt_rec,
                        P->alt_index_mem, P->grad_mem})
            if (p) (void)hipFree(p);
    }
    if (P->thread_scratch) (void)hipFree(P->thread_scratch);
    delete P;
}

const char *lm_status_string(int code)
{
    switch (code) {
    case LM_OK: return "ok";
    case LM_ERR_INVALID_ARG: return "invalid argument";
    case LM_ERR_BAD_LATTICE: return "strut endpoint out of range";
    case LM_ERR_CAPACITY: return "buffer or workspace too small";
    case LM_ERR_UNSUPPORTED: return "size or feature not supported (by this library or this workspace)";
    case LM_ERR_HIP: return "HIP runtime error";
    case LM_ERR_STATE: return "call out of order";
    case LM_ERR_INTERNAL: return "workspace could not be sized";
    case LM_ERR_IO: return "file could not be written";
    case LM_ERR_RADIUS_MISMATCH: return "end radii at a node differ";
    default: return "unknown status";
    }
}

}  // extern "C"

// ---- sink mode without allocation ------------------------------------------
// Device memory of lm_forward_sink_static: the whole plan (adjacency, counts,
// node lists, slots and node records) is carved from this array.  Every GPU
// the library runs on holds its own copy, at its own address, until the
// process ends.  In host code `scratch` only stands for the symbol: its device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[LM_STATIC_SCRATCH_BYTES];

__global__ void lm_k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up at the first
// call on that device).
int static_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LM_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return LM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LM_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LM_OK;
}

// Clears n 32-bit words with a kernel (no memset node).
int fill_u32(void *p, int64_t n, hipStream_t st)
{
    if (n <= 0) return LM_OK;
    lm_k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>((uint32_t *)p, 0u, n);
    return hipGetLastError() == hipSuccess ? LM_OK : LM_ERR_HIP;
}

}  // namespace

extern "C" {

int lm_static_scratch_size(int64_t n_nodes, int64_t n_struts, int k, size_t *bytes)
{
    if (!bytes || k < 3 || k > 4096) return LM_ERR_INVALID_ARG;
    lm_options o;
    o.flags = LM_WS_SINK;
    o.k_max = k;
    o.record_bytes = 0;
    o.max_parts = 0;
    return lm_workspace_size(n_nodes, n_struts, &o, bytes);
}

int lm_forward_sink_static(const lm_lattice *lat, int k, uint64_t *d_words, void *stream)
{
    if (!d_words || k < 3 || k > 4096) return LM_ERR_INVALID_ARG;
    int rc = check_lattice(lat);
    if (rc) return rc;
    size_t need = 0;
    if ((rc = lm_static_scratch_size(lat->n_nodes, lat->n_struts, k, &need))) return rc;
    if (need > (size_t)LM_STATIC_SCRATCH_BYTES) return LM_ERR_CAPACITY;  // before any device call
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = lat->n_nodes;
    if (N == 0) {
        if ((rc = fill_u32(d_words, 2 * LM_SINK_WORDS, st))) return rc;
        return hipStreamSynchronize(st) == hipSuccess ? LM_OK : LM_ERR_HIP;
    }
    void *base = nullptr;
    if ((rc = static_scratch(&base))) return rc;
    // a plan on the stack, every device buffer carved from the array
    lm_plan P{};  // value-initialised: every device pointer starts null
    init_plan(&P, lat, stream);
    P.caller_ws = true;
    P.ws_flags = LM_WS_SINK;
    lm_options o;
    o.flags = LM_WS_SINK;
    o.k_max = k;
    o.record_bytes = 0;
    o.max_parts = 0;
    ws_layout(&P, base, lat->n_nodes, lat->n_struts, o);
    // the array keeps the previous call's contents: clear what the sink
    // range expects at zero (node marks, slots, the range's failure flag)
    if ((rc = fill_u32(P.sk_mark, N + 1, st)) ||
        (rc = fill_u32(P.sk_slots, 2 * lm::sink_slots_words(), st)) || (rc = fill_u32(P.sk_fail, 1, st)))
        return rc;
    if ((rc = first_prepare(&P))) return rc;  // synchronises; LM_ERR_BAD_LATTICE
    if ((rc = fill_u32(P.w.flags, 3, st))) return rc;
    lm::SinkOut so{0, 0, P.sk_slots, nullptr, nullptr, nullptr};
    if ((rc = sink_range(&P, k, 0, 0, N, 4, 8, so, d_words))) return rc;
    int32_t fail = 0;
    if (hipMemcpyAsync(&fail, P.sk_fail, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return LM_ERR_HIP;
    return fail ? LM_ERR_CAPACITY : LM_OK;
}

}  // extern "C"
