/*
 * latmesh: meta-meshing and arc-subdivision triangulation of strut lattices
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Zou & Gao, "Warp-centric GPU meta-meshing and fast triangulation of
 * billion-scale lattice structures".  A lattice is a set of nodes (centre,
 * nodal-sphere radius) joined by struts; every strut is the round cone tangent
 * to the spheres of its two end nodes (Sec. 4.1).  Around each node the
 * incident struts are intersected pairwise on auxiliary planes into elliptic
 * arcs (Sec. 4.3.1, Eq. 7), trimmed against the node's other struts
 * (Eqs. 8-9), and assembled into the node's meta-mesh: vertices, arcs, one
 * arc loop per strut end and hole contours bounded by circular arcs.  The
 * meta-mesh is then subdivided at k segments per full turn (Eqs. 11-12), each
 * strut band is triangulated between its two end loops and each hole is
 * filled by a fan from its projected barycentre (Sec. 5, Eq. 13).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are DEVICE pointers owned by the caller; the library
 *     reads inputs and writes outputs through them and keeps no reference
 *     after the call returns, except that a plan keeps its lattice pointers
 *     until lm_plan_destroy (the caller must keep them alive and unchanged).
 *   - Work is ordered on the plan's HIP stream.  Calls that return host
 *     values (lm_count, lm_read_totals) synchronise that stream.
 *   - Functions return LM_OK (0) or a negative LM_ERR_* code and never throw.
 *     Problems with single nodes do not fail a call: they are reported per
 *     node as LM_NODE_* bits and such nodes emit nothing.
 *   - A plan is not thread safe; use one plan per host thread.
 */
#ifndef LATMESH_H
#define LATMESH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define LM_OK 0
#define LM_ERR_INVALID_ARG (-1)    /* null pointer, negative size, bad k */
#define LM_ERR_BAD_LATTICE (-2)    /* strut endpoint index outside [0, n_nodes) */
#define LM_ERR_CAPACITY (-3)       /* an output buffer is smaller than the totals */
#define LM_ERR_UNSUPPORTED (-4)    /* size beyond what this library handles */
#define LM_ERR_HIP (-5)            /* a HIP runtime call failed */
#define LM_ERR_STATE (-6)          /* call out of order (e.g. fill before count) */
#define LM_ERR_INTERNAL (-7)       /* the workspace could not be sized */
#define LM_ERR_IO (-8)             /* a file could not be opened or written */
#define LM_ERR_RADIUS_MISMATCH (-9) /* the end radii of a node's struts differ */

/* ---- per-node status bits (node_status output) ------------------------- */
#define LM_NODE_INVALID_STRUT 1u   /* |r_a - r_b| >= length, zero length or self loop */
#define LM_NODE_NON_ELLIPTIC 2u    /* a seam plane cuts a cone in a non-ellipse */
#define LM_NODE_LOOP 4u            /* a strut end loop is not one closed curve
                                      monotone in the strut angle */
#define LM_NODE_TOPOLOGY 8u        /* arc/vertex incidence or Euler check failed
                                      (e.g. an annular hole), or no hole-fan apex */
#define LM_NODE_ISOLATED 16u       /* no incident strut */
#define LM_NODE_VALENCE 32u        /* more incident struts than this library handles (64) */
#define LM_NODE_DUPLICATE 64u      /* two struts join the same pair of nodes */
#define LM_NODE_CAPACITY 128u      /* per-node arc / vertex / piece capacity exceeded */

/* Lattice: n_nodes nodes with centre (x, y, z) and nodal-sphere radius
 * radius (FP32, one value per node, Sec. 4.1: struts are tangent to the nodal
 * spheres), and n_struts struts joining nodes strut_a[i] and strut_b[i].
 * Struct of arrays, device memory, caller owned. */
typedef struct lm_lattice {
    int64_t n_nodes;
    int64_t n_struts;
    const float *d_x, *d_y, *d_z, *d_radius; /* [n_nodes] */
    const int32_t *d_strut_a, *d_strut_b;    /* [n_struts] */
} lm_lattice;

/* Sizes produced by lm_count for resolution k. */
typedef struct lm_totals {
    int64_t n_vertices;      /* meta-mesh vertices (arc junctions) */
    int64_t n_arcs;          /* meta-mesh arcs */
    int64_t n_holes;         /* hole contours */
    int64_t n_mesh_vertices; /* triangle-mesh vertices */
    int64_t n_triangles;     /* = n_band_triangles + n_fan_triangles */
    int64_t n_band_triangles;
    int64_t n_fan_triangles;
    int64_t n_record_bytes;  /* internal: workspace bytes of the node records */
    int64_t n_bad_nodes;     /* nodes with a nonzero status */
    int64_t n_skipped_struts;/* struts not triangulated (an end node is bad) */
    int64_t n_fp64_nodes;    /* nodes meshed in FP64 (see lm_set_precision) */
} lm_totals;

/* Output buffers for lm_fill (device memory, caller owned).
 *
 * Mesh (required):
 *   d_mesh_xyz [cap_mesh_vertices][3] FP32 absolute vertex positions;
 *   d_tri      [cap_triangles][3] int32 vertex indices, counter-clockwise seen
 *              from outside.  Order: the band triangles of strut 0, 1, ...,
 *              then the hole-fan triangles of node 0, 1, ...
 *   Mesh vertices are numbered node by node; within a node: meta-vertices
 *   (by name), then the interior subdivision points of each arc (arcs in
 *   meta-mesh order, points from the endpoint with the smaller name), then
 *   one hole centre per hole contour.
 *
 * Meta-mesh (optional; pass NULL to skip), positions local to their node
 * (add the node centre for absolute coordinates):
 *   d_vert_name [cap_vertices] uint32 name (p<<24 | q<<16 | r<<8 | root):
 *               the vertex is where struts p<q<r tie (label 0 = nodal sphere,
 *               labels 1..v = incident struts in increasing strut id), root
 *               = rank of the two tie points along (g_p-g_q)x(g_p-g_r);
 *               r = 255 marks the start point of an arc that is a whole conic;
 *   d_vert_xyz  [3][cap_vertices] FP32 (field-major);
 *   d_arc_f32   [11][cap_arcs] FP32 field-major: o.xyz, a.xyz, b.xyz, t1, t2
 *               with x(t) = o + a sin t + b cos t for t in [t1, t2] (Eq. 1,
 *               a = semi-major, b = semi-minor axis);
 *   d_arc_u32   [3][cap_arcs] uint32 field-major: (p | q<<8 | whole<<16),
 *               (start vertex | end vertex<<16) as node-local vertex indices
 *               (start = end at t1 / t2), node index;
 *   d_node_off  [5][n_nodes+1] int64 field-major exclusive prefix sums of the
 *               per-node counts: vertices, arcs, holes, mesh vertices, fan
 *               triangles;
 *   d_node_status [n_nodes] uint8 LM_NODE_* bits;
 *   d_strut_off [n_struts+1] int64 exclusive prefix sum of the band
 *               triangles per strut (0 for a strut with a bad end node).
 */
typedef struct lm_outputs {
    float *d_mesh_xyz;
    int32_t *d_tri;
    int64_t cap_mesh_vertices;
    int64_t cap_triangles;
    uint32_t *d_vert_name;
    float *d_vert_xyz;
    int64_t cap_vertices;
    float *d_arc_f32;
    uint32_t *d_arc_u32;
    int64_t cap_arcs;
    int64_t *d_node_off;
    uint8_t *d_node_status;
    int64_t *d_strut_off;
} lm_outputs;

typedef struct lm_plan lm_plan;

/* Create a plan for one lattice: validates strut indices (A0), builds the
 * node adjacency with incident struts in increasing strut id (A1).  The plan
 * allocates its own device workspace (about 110 bytes per node plus 80 bytes
 * per strut) and, at the first lm_count or lm_forward, the node-record space
 * (each meshed node's meta-mesh and strut end loops: about 1.2 kB per node
 * plus 8 bytes per loop sample, about 2.5 kB per node of the BCC lattice at
 * k = 16); sink mode, batched parts, the adjoint and re-triangulation
 * allocate their scratch at their first call (lm_plan_create_in allocates
 * nothing).  stream is a hipStream_t (NULL = default stream).  On success
 * *plan is set; on error it is NULL.  Returns LM_ERR_BAD_LATTICE for
 * out-of-range endpoints, LM_ERR_UNSUPPORTED if n_nodes or n_struts is 2^31
 * or more. */
int lm_plan_create(lm_plan **plan, const lm_lattice *lat, void *stream);

/* ---- caller-owned device memory ------------------------------------------
 * A plan made by lm_plan_create_in takes all of its device memory from one
 * caller buffer sized by lm_workspace_size and allocates no device memory
 * afterwards: a call that needs more node-record space than was sized
 * returns LM_ERR_CAPACITY (lm_count: with the needed bytes in
 * n_record_bytes), one that needs a part not requested in opt->flags returns
 * LM_ERR_UNSUPPORTED, writing nothing.  (lm_write_stl, which takes no plan,
 * allocates its own staging buffers.) */
#define LM_WS_SINK 1      /* lm_forward_sink and lm_batched */
#define LM_WS_GRADIENT 2  /* lm_loss and lm_backward */
#define LM_WS_RETRI 4     /* lm_retriangulate (a second node-record space) */

typedef struct lm_options {
    int32_t flags;        /* LM_WS_* */
    int32_t k_max;        /* resolution the node-record space is sized for when record_bytes is 0 */
    int64_t record_bytes; /* node-record space in bytes; 0: an estimate for the whole lattice at k_max
                             (sink-mode chunks need only their nodes' share) */
    int64_t max_parts;    /* most parts of one lm_batched call (with LM_WS_SINK) */
} lm_options;

/* Bytes of device memory a plan for n_nodes nodes and n_struts struts needs
 * with options opt (NULL: no optional parts, records for k = 16).  Returns
 * LM_ERR_INVALID_ARG for negative sizes, k_max outside 3..4096 or a negative
 * record_bytes / max_parts, LM_ERR_UNSUPPORTED for 2^31 nodes or struts or
 * more. */
int lm_workspace_size(int64_t n_nodes, int64_t n_struts, const lm_options *opt, size_t *bytes);

/* lm_plan_create with all device memory in d_workspace (device, 256-byte
 * aligned, at least lm_workspace_size(lat->n_nodes, lat->n_struts, opt)
 * bytes, owned by the caller and kept alive until lm_plan_destroy).
 * LM_ERR_CAPACITY if workspace_bytes is too small. */
int lm_plan_create_in(lm_plan **plan, const lm_lattice *lat, const lm_options *opt, void *d_workspace,
                      size_t workspace_bytes, void *stream);

/* Per-strut end radii (Sec. 4.1: every strut is the cone tangent to the
 * nodal spheres of its ends, so all struts meeting at a node have the same
 * radius there).  d_end_radius [n_struts][2] (device) holds the radius of
 * strut i at strut_a[i] and at strut_b[i]; the node radius is the mean of
 * its incident struts' end radii (taken in increasing strut id), written to
 * d_radius [n_nodes] (device; 0 for a node without struts), and the plan is
 * created for the lattice with those radii (lat->d_radius is not read; the
 * plan keeps d_radius).  If at some node two end radii differ by more than
 * rel_tol times their mean, no plan is made and LM_ERR_RADIUS_MISMATCH is
 * returned (d_radius then holds the means); *n_mismatch (host, may be NULL)
 * receives the number of such nodes.  Gradients with respect to end radii:
 * lm_end_radius_gradient.  Synchronises the stream. */
int lm_plan_create_end_radii(lm_plan **plan, const lm_lattice *lat, const float *d_end_radius, float rel_tol,
                             float *d_radius, int64_t *n_mismatch, void *stream);

/* Maps a gradient with respect to node radii (lm_backward's d_grad_radius)
 * to the end radii of a plan made by lm_plan_create_end_radii: the end of
 * strut i at node n gets d_grad_radius[n] / (struts at n), the derivative of
 * the mean.  d_grad_end [n_struts][2] (device).  Asynchronous. */
int lm_end_radius_gradient(lm_plan *plan, const float *d_grad_radius, float *d_grad_end);

/* Redo the validation and adjacency build of lm_plan_create on the device,
 * asynchronously (the lattice arrays may have changed in place; the sizes
 * may not).  An out-of-range endpoint is reported by the next
 * lm_read_totals as LM_ERR_BAD_LATTICE. */
int lm_prepare(lm_plan *plan);

/* Meta-mesh every node and size the triangulation at k segments per full
 * turn (Eq. 11 with step 2 pi / k; 3 <= k <= 4096): per-node arcs,
 * vertices, holes, end loops and counts, prefix sums.  Each node's result is
 * kept in the plan's node-record space for lm_fill (the space grows, and the
 * pass runs again, if it was too small).  Synchronises the stream and writes
 * the totals to *totals (host memory).  Re-callable with another k on the
 * same plan. */
int lm_count(lm_plan *plan, int k, lm_totals *totals);

/* Write the meta-mesh and the triangle mesh for the k of the last lm_count
 * (A9, B1-B3) from the node records.  Asynchronous on the plan's stream.
 * Returns LM_ERR_CAPACITY (writing nothing) if a required buffer is smaller
 * than the totals, LM_ERR_STATE if lm_count has not run. */
int lm_fill(lm_plan *plan, const lm_outputs *out);

/* lm_count and lm_fill without the host synchronisation: sizes are taken on
 * the device; if an output or the node-record space is too small nothing is
 * written and lm_read_totals reports LM_ERR_CAPACITY afterwards.  For
 * repeated runs with buffers (and record space) sized by an earlier
 * lm_count at the same or a larger k. */
int lm_forward(lm_plan *plan, int k, const lm_outputs *out);

/* Multi-resolution re-triangulation (Alg. 1 keeps the meta-mesh apart from
 * its subdivision; Eqs. 11-13).  Subdivide the meta-mesh of the last
 * lm_count or lm_forward again at k segments per full turn (3 <= k <= 4096)
 * and write the triangle mesh, without re-solving any node: vertices, arcs
 * and holes are read from the stored node records and only the arc
 * subdivision, the end loops, the fans and the strut bands are redone.  The
 * result equals lm_forward at k on the same lattice except for nodes whose
 * status depends on k (a loop or subdivision failure at one of the two
 * resolutions).  The meta-mesh stays in the plan: any number of calls may
 * follow, each from the same meta-mesh.  The new records go to a second
 * record space held by the plan (allocated at the first call; about the
 * size of the first at the same k); lm_loss and lm_backward then act on the
 * re-triangulated mesh.  lm_fill returns LM_ERR_STATE until the next
 * lm_count.  Asynchronous; read the totals with lm_read_totals, which
 * returns LM_ERR_CAPACITY if a buffer was too small (then nothing usable
 * was written).  Returns LM_ERR_STATE if no meta-mesh is held (lm_count or
 * lm_forward has not run, or lm_forward_sink, lm_batched or
 * lm_set_precision ran after it). */
int lm_retriangulate(lm_plan *plan, int k, const lm_outputs *out);

/* Synchronise the stream and return the totals of the last lm_forward,
 * lm_retriangulate or lm_count; LM_ERR_CAPACITY if that call skipped
 * writes. */
int lm_read_totals(lm_plan *plan, lm_totals *totals);

/* Mixed precision.  Nodes are meshed in FP32; a node is meshed again in
 * FP64 when an FP32 consistency check fails or when one of its vertices has
 * a condition number above kappa_max (kappa = |n1||n2||n3| / |det(n1,n2,n3)|
 * for the normals of the three surfaces meeting there, which bounds how much
 * FP32 rounding is amplified in the vertex position).  Default 32; 0 meshes
 * every node in FP64.  Invalidates the last lm_count. */
int lm_set_precision(lm_plan *plan, float kappa_max);

/* Scheduling of the FP32 node pass of lm_count and lm_forward.
 * LM_SCHEDULE_WAVE (default): a node per group of lanes of a wave, lanes
 * over its conics and samples, nodes bucketed by valence, per-node scratch in
 * LDS (the paper's warp-centric design, Sec. 4.3, on 64-lane waves).
 * LM_SCHEDULE_THREAD: an ablation of it — one lane per node, nodes in id
 * order without buckets, per-node scratch in global memory (allocated at the
 * first use, about 3 GB) — the thread-centric design the paper measures
 * against.  Both give identical results.  Re-triangulation, sink mode and
 * batched parts always use the wave schedule. */
#define LM_SCHEDULE_WAVE 0
#define LM_SCHEDULE_THREAD 1
int lm_set_schedule(lm_plan *plan, int schedule);

/* Profiling: when on, every library call records HIP events on the plan's
 * stream around its phases; lm_get_profile synchronises the stream and
 * returns, per phase, the summed milliseconds and the number of timed calls
 * since the last lm_get_profile.  Phases (n >= 8): 0 lm_prepare, 1 FP32
 * meta-meshing of every node, 2 FP64 meta-meshing of the handed-over nodes,
 * 3 band counts + prefix sums + totals, 4 expansion of the node results into
 * the meta-mesh, mesh vertices and hole fans, 5 strut bands, 6 lm_loss,
 * 7 lm_backward. */
int lm_set_profiling(lm_plan *plan, int on);
int lm_get_profile(lm_plan *plan, double *ms, int64_t *calls, int n);

/* ---- sink mode: chunked meshing reduced to counts and hashes ---------- */

/* Words per chunk written by lm_forward_sink. */
#define LM_SINK_WORDS 8

/* Mesh the lattice at resolution k in chunks of chunk_nodes consecutive node
 * ids and, instead of storing the mesh, write per chunk LM_SINK_WORDS
 * uint64 words to d_out[chunk][LM_SINK_WORDS] (device):
 *   0 triangles (hole fans of the chunk's nodes, bands of struts whose lower
 *     node id is in the chunk), 1 sum of triangle keys, 2 mesh vertices of
 *     the chunk's nodes, 3 sum of vertex keys, 4..6 sums of round(2^20 x),
 *     round(2^20 y), round(2^20 z) over those vertices (two's complement),
 *     7 nodes of the chunk without a mesh (nonzero status).
 * A mesh vertex is named vid = node << 21 | node-local index (the index of
 * the stored mode); a triangle's key is m(m(m(v0 + G) ^ v1) ^ v2) with its
 * vids rotated so that the smallest comes first (orientation kept), a
 * vertex's key m(m(m(vid) ^ (bits(x) | bits(y) << 32)) ^ bits(z)) over its
 * FP32 position, m the SplitMix64 finaliser and G = 0x9E3779B97F4A7C15.
 * Sums are modulo 2^64, so totals over chunks are chunking independent.
 * Each chunk also meshes the higher-id neighbours of its nodes outside it
 * (for the bands; with node ids numbered in spatial layers this halo is a
 * thin shell).  The node pass hashes vertices and fans itself and keeps
 * only the strut end loops for the bands.  Chunks run back to back without
 * host synchronisation; the call synchronises once at the end (and runs a
 * chunk again, with more record space, if its records did not fit; with a
 * caller-owned workspace that is LM_ERR_CAPACITY instead).  LM_ERR_CAPACITY
 * if n_chunks_cap < ceil(n_nodes / chunk_nodes); LM_ERR_UNSUPPORTED for a
 * caller-owned workspace without LM_WS_SINK.  The node records then hold
 * the last chunk only: lm_fill and lm_backward need a new lm_count. */
int lm_forward_sink(lm_plan *plan, int k, int64_t chunk_nodes, uint64_t *d_out, int64_t n_chunks_cap);

/* ---- sink mode without allocation ---------------------------------------
 * For callers that cannot allocate device memory (tight serving loops, code
 * that must not call hipMalloc): one lattice meshed in sink mode as a single
 * chunk, every device buffer (adjacency, node lists, hash slots, node records)
 * carved from a fixed array that the library holds in device memory,
 * LM_STATIC_SCRATCH_BYTES on each GPU it runs on, kept until the process ends.
 * Nothing is allocated, on the device or the host.  The BCC lattice of 24^3
 * cells (29,449 nodes, 110,592 struts) at k = 16 needs 108 MiB;
 * lm_static_scratch_size gives the exact need of a lattice. */
#define LM_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

/* Bytes of the fixed array that lm_forward_sink_static needs for a lattice of
 * n_nodes nodes and n_struts struts at resolution k (3..4096).  Host only. */
int lm_static_scratch_size(int64_t n_nodes, int64_t n_struts, int k, size_t *bytes);

/* The words of lm_forward_sink over the whole lattice as one chunk
 * (d_words[LM_SINK_WORDS], device; see lm_forward_sink), computed without a
 * plan and without allocating: the same validation, adjacency, node pass and
 * band hashing, with the fixed array as workspace.  stream is a hipStream_t
 * of the current device (whose copy of the array is used).  Returns
 * LM_ERR_CAPACITY, before any device work, when the lattice needs more than
 * LM_STATIC_SCRATCH_BYTES (or, after the pass, if its node records did not
 * fit); LM_ERR_BAD_LATTICE for out-of-range endpoints; the checks of
 * lm_plan_create otherwise.  A lattice without nodes gives zero words.
 * Synchronises the stream (so it cannot be captured into a graph).  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU (two
 * host threads, or two streams) race and must be serialised by the caller. */
int lm_forward_sink_static(const lm_lattice *lat, int k, uint64_t *d_words, void *stream);

/* ---- batched parts -------------------------------------------------------- */

/* Work mapping of lm_batched: nodes of valence <= v_four_per_wave (at most 4)
 * go four to a wave, up to v_two_per_wave (at most 8) two to a wave, the rest
 * up to 16 one to a wave, above that four waves to a node; group_nodes whole
 * parts' worth of nodes (about) share one node pass (0: all parts in one
 * pass when their records fit the device memory, else the fewest groups
 * that fit). */
typedef struct lm_tuning {
    int32_t v_four_per_wave;
    int32_t v_two_per_wave;
    int64_t group_nodes;
} lm_tuning;

/* Many lattice parts in one plan: part p is the node range
 * [part_off[p], part_off[p+1]) of the plan's lattice (host arrays; part_off[0]
 * = 0, part_off[n_parts] = n_nodes; struts should join nodes of one part) and
 * is meshed at its own resolution part_k[p] (3..4096).  The nodes of all
 * parts (of a group, when tune->group_nodes splits them) are meshed by one
 * persistent launch per valence class that takes its work from a global
 * queue ordered by valence class, whatever the part; then one launch hashes
 * the bands of all their struts.  Output per part, in sink mode:
 * d_out[p][LM_SINK_WORDS] (device; the words of lm_forward_sink, counted per
 * part: a band goes to the part of its lower node; vertex ids use node ids
 * local to the part, so a part's words equal those of lm_forward_sink on
 * the part alone).  tune may be NULL (limits 4 and 8, automatic groups).
 * Synchronises the stream once (again per group whose records did not fit
 * and is run a second time).  With a caller-owned workspace: needs
 * LM_WS_SINK and n_parts <= max_parts. */
int lm_batched(lm_plan *plan, int64_t n_parts, const int64_t *part_off, const int32_t *part_k,
               const lm_tuning *tune, uint64_t *d_out);

/* ---- adjoint at fixed topology (gradients of a mesh loss) ------------- */

/* Weights of the loss L = area * Area + volume * Vol + sq_norm * sum |v|^2
 * over the triangle mesh; Vol is the signed volume enclosed about the point
 * p0 (sum over triangles of (a-p0) . ((b-p0) x (c-p0)) / 6). */
typedef struct lm_loss_weights {
    float area, volume, sq_norm;
    float p0[3];
} lm_loss_weights;

/* Loss terms of the mesh written by the last lm_fill / lm_forward into
 * `out` (its d_mesh_xyz and d_tri): d_terms (device, 3 doubles) receives
 * Area, Vol and sum |v|^2 (unweighted), d_dl_dx (device, [cap_mesh_vertices]
 * [3] FP32) receives dL/dx for every mesh vertex (overwritten).  The terms
 * are summed per node and then in a fixed order (bit-reproducible).
 * Returns LM_ERR_CAPACITY, launching nothing, when the totals of the last
 * lm_count exceed out's capacities; after lm_forward (totals on the device)
 * the kernels check and write nothing instead, and lm_read_totals then
 * returns LM_ERR_CAPACITY (also when that pass itself skipped writes).
 * LM_ERR_UNSUPPORTED for a caller-owned workspace without LM_WS_GRADIENT.
 * Asynchronous.  Not a step of the method: a convenience loss for the
 * adjoint. */
int lm_loss(lm_plan *plan, const lm_outputs *out, const lm_loss_weights *w, double *d_terms, float *d_dl_dx);

/* Gradient of a loss with respect to the node centres and radii, given its
 * gradient d_dl_dx ([n_mesh_vertices][3], device) with respect to the mesh
 * vertices of the last lm_fill / lm_forward on this plan, at that pass's
 * topology (labels, arcs, segment counts and triangles fixed; every mesh
 * vertex moves with the inputs as the method defines it: vertices as triple
 * ties, Eq. 12 interior points, Eq. 13 hole centres).  Writes
 * d_grad_xyz [n_nodes][3] and d_grad_radius [n_nodes] (device, FP32;
 * nodes with a nonzero status contribute nothing).  Each node's adjoint and
 * the parts it contributes to its neighbours are written per node and per
 * strut end and summed in adjacency order, so the result is bit-reproducible.
 * The plan must not have been counted again since that pass; if that pass
 * (or lm_loss) skipped writes for lack of capacity, zeros are written.
 * LM_ERR_UNSUPPORTED for a caller-owned workspace without LM_WS_GRADIENT.
 * Asynchronous. */
int lm_backward(lm_plan *plan, const float *d_dl_dx, float *d_grad_xyz, float *d_grad_radius);

/* Release the plan and its workspace (synchronises its stream). */
void lm_plan_destroy(lm_plan *plan);

/* Text for an LM_OK / LM_ERR_* code (static storage). */
const char *lm_status_string(int code);

/* ---- lossy arc codec ---------------------------------------------------- */

/* Compressed meta-mesh arcs (Sec. 4.2.1): 128 bits per arc, or the arc kept
 * whole when it falls outside the format's ranges.  All device memory,
 * caller-owned. */
typedef struct lm_arc_codes {
    uint32_t *d_codes;         /* [cap_arcs][4]; a fallback arc's code holds its slot */
    uint32_t *d_fallback_mask; /* [(cap_arcs + 31) / 32], bit j: arc j kept whole */
    float *d_fallback;         /* [cap_fallback][11] arcs kept whole (any order) */
    int64_t cap_arcs;
    int64_t cap_fallback;
} lm_arc_codes;

/* Encode n_arcs meta-mesh arcs given as lm_outputs arrays (d_arc_f32
 * [11][ld] o, a, b, t1, t2 node-local; d_arc_u32 [3][ld] with p | q << 8 in
 * row 0 and the node in row 2) of the plan's lattice, whose adjacency must
 * be the one the arcs were made with (lm_prepare state).  The semi-major
 * axis a and the centre o are kept as spherical coordinates (12-bit radius,
 * 15-bit polar angle, 16-bit azimuth; a in [r_min, 4 r_max], o within
 * r_max), the semi-minor axis b as its 12-bit length in [0.1 r_min, r_max]
 * (its direction is a x d / |a x d|, d the strut direction for a tangency
 * circle or the normal of the seam plane (g_p - g_q) / |g_p - g_q| for an
 * ellipse), t1 on 15 bits over [0, 2 pi) and t2 - t1 on 15 bits over
 * [0, 2 pi].  r_min, r_max: the smallest and largest node radius.  Decoded
 * points lie within Eq. 5's 8.69e-4 r_max of the arc's points at the same t.
 * Synchronises the stream; *n_fallback (host) receives the number of arcs
 * kept whole.  Returns LM_ERR_CAPACITY if that number exceeds cap_fallback
 * (then the codes of the excess arcs are unusable). */
int lm_arc_encode(lm_plan *plan, const float *d_arc_f32, const uint32_t *d_arc_u32, int64_t n_arcs, int64_t ld,
                  float r_min, float r_max, const lm_arc_codes *codes, int64_t *n_fallback);

/* Decode the first n_arcs codes into d_arc_f32_out [11][ld_out] (same
 * fields as lm_outputs.d_arc_f32), with d_arc_u32 and r_min, r_max as given
 * to lm_arc_encode.  Asynchronous. */
int lm_arc_decode(lm_plan *plan, const lm_arc_codes *codes, const uint32_t *d_arc_u32, int64_t n_arcs, int64_t ld,
                  float r_min, float r_max, float *d_arc_f32_out, int64_t ld_out);

/* ---- STL output ---------------------------------------------------------- */

/* lm_write_stl flags */
#define LM_STL_FSYNC 1  /* fsync the file before returning (time includes the disk) */

/* What one lm_write_stl call moved and where its time went. */
typedef struct lm_stl_stats {
    int64_t n_triangles;
    int64_t n_bytes;          /* file size: 84 + 50 n_triangles */
    int64_t n_chunks;
    int64_t chunk_triangles;  /* triangles per chunk (whole blocks of 256) */
    double seconds;           /* wall time of the call */
    double encode_ms;         /* device time of the encode kernels, summed */
    double copy_ms;           /* device-to-host copy time, summed */
    double write_s;           /* host time in write() (and fsync) */
} lm_stl_stats;

/* Binary STL of an indexed triangle mesh on the device (the output stage of
 * the paper's asynchronous pipeline, Sec. 4.2.2, with 50-byte triangle
 * records and the batch sized by the I/O buffer as in Eq. 6).
 * d_mesh_xyz [n_mesh_vertices][3] FP32 and d_tri [n_triangles][3] int32 are
 * device pointers (e.g. an lm_outputs after lm_forward; the call is ordered
 * after earlier work on `stream`).  The file gets an 80-byte header, the
 * count, and per triangle the unit normal of (v1 - v0) x (v2 - v0) (zero if
 * degenerate), the three vertices and a zero attribute word.  The mesh goes
 * out in chunks of about chunk_bytes (at least 12,800): the device encodes
 * chunk i on `stream` while chunk i-1 is copied on a second stream into
 * pinned host memory and written to the file by the calling thread, so
 * encoding, the PCIe copy and the disk overlap.  path NULL runs the pipeline without a
 * file (to time the device and PCIe part).  The call allocates two device
 * and two pinned host buffers of chunk_bytes, frees them before returning,
 * and synchronises the stream.  Returns LM_ERR_INVALID_ARG if a triangle
 * index is outside [0, n_mesh_vertices) (the file is then incomplete),
 * LM_ERR_UNSUPPORTED for 2^32 or more triangles, LM_ERR_IO if the file
 * cannot be written.  stats may be NULL. */
int lm_write_stl(const float *d_mesh_xyz, int64_t n_mesh_vertices, const int32_t *d_tri, int64_t n_triangles,
                 const char *path, int64_t chunk_bytes, int flags, void *stream, lm_stl_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* LATMESH_H */
