"""ctypes binding of liblatmesh.so (include/latmesh.h) plus a thin torch-side
helper that allocates device buffers.  All computation happens in the HIP
kernels of the library; this module only marshals arguments.  There is no
CPU fallback: if the library or a GPU is missing, calls raise."""

from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblatmesh.so")

LM_OK = 0
LM_ERR_INVALID_ARG = -1
LM_ERR_BAD_LATTICE = -2
LM_ERR_CAPACITY = -3
LM_ERR_UNSUPPORTED = -4
LM_ERR_HIP = -5
LM_ERR_STATE = -6
LM_ERR_INTERNAL = -7
LM_ERR_IO = -8
LM_ERR_RADIUS_MISMATCH = -9

LM_WS_SINK = 1
LM_WS_GRADIENT = 2
LM_WS_RETRI = 4

LM_NODE_INVALID_STRUT = 1
LM_NODE_NON_ELLIPTIC = 2
LM_NODE_LOOP = 4
LM_NODE_TOPOLOGY = 8
LM_NODE_ISOLATED = 16
LM_NODE_VALENCE = 32
LM_NODE_DUPLICATE = 64
LM_NODE_CAPACITY = 128

# every function the header declares (checked by the CPU tests)
EXPORTS = (
    "lm_plan_create",
    "lm_workspace_size",
    "lm_plan_create_in",
    "lm_plan_create_end_radii",
    "lm_end_radius_gradient",
    "lm_prepare",
    "lm_count",
    "lm_fill",
    "lm_forward",
    "lm_retriangulate",
    "lm_read_totals",
    "lm_set_precision",
    "lm_set_schedule",
    "lm_set_profiling",
    "lm_get_profile",
    "lm_forward_sink",
    "lm_static_scratch_size",
    "lm_forward_sink_static",
    "lm_batched",
    "lm_loss",
    "lm_backward",
    "lm_write_stl",
    "lm_arc_encode",
    "lm_arc_decode",
    "lm_plan_destroy",
    "lm_status_string",
)


class lm_lattice(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int64),
        ("n_struts", ctypes.c_int64),
        ("d_x", ctypes.c_void_p),
        ("d_y", ctypes.c_void_p),
        ("d_z", ctypes.c_void_p),
        ("d_radius", ctypes.c_void_p),
        ("d_strut_a", ctypes.c_void_p),
        ("d_strut_b", ctypes.c_void_p),
    ]


class lm_options(ctypes.Structure):
    _fields_ = [
        ("flags", ctypes.c_int32),
        ("k_max", ctypes.c_int32),
        ("record_bytes", ctypes.c_int64),
        ("max_parts", ctypes.c_int64),
    ]


class lm_arc_codes(ctypes.Structure):
    _fields_ = [
        ("d_codes", ctypes.c_void_p),
        ("d_fallback_mask", ctypes.c_void_p),
        ("d_fallback", ctypes.c_void_p),
        ("cap_arcs", ctypes.c_int64),
        ("cap_fallback", ctypes.c_int64),
    ]


class lm_stl_stats(ctypes.Structure):
    _fields_ = [
        ("n_triangles", ctypes.c_int64),
        ("n_bytes", ctypes.c_int64),
        ("n_chunks", ctypes.c_int64),
        ("chunk_triangles", ctypes.c_int64),
        ("seconds", ctypes.c_double),
        ("encode_ms", ctypes.c_double),
        ("copy_ms", ctypes.c_double),
        ("write_s", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


LM_STL_FSYNC = 1


_TOTAL_FIELDS = [
    "n_vertices",
    "n_arcs",
    "n_holes",
    "n_mesh_vertices",
    "n_triangles",
    "n_band_triangles",
    "n_fan_triangles",
    "n_record_bytes",
    "n_bad_nodes",
    "n_skipped_struts",
    "n_fp64_nodes",
]


class lm_totals(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in _TOTAL_FIELDS]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f in _TOTAL_FIELDS}


class lm_outputs(ctypes.Structure):
    _fields_ = [
        ("d_mesh_xyz", ctypes.c_void_p),
        ("d_tri", ctypes.c_void_p),
        ("cap_mesh_vertices", ctypes.c_int64),
        ("cap_triangles", ctypes.c_int64),
        ("d_vert_name", ctypes.c_void_p),
        ("d_vert_xyz", ctypes.c_void_p),
        ("cap_vertices", ctypes.c_int64),
        ("d_arc_f32", ctypes.c_void_p),
        ("d_arc_u32", ctypes.c_void_p),
        ("cap_arcs", ctypes.c_int64),
        ("d_node_off", ctypes.c_void_p),
        ("d_node_status", ctypes.c_void_p),
        ("d_strut_off", ctypes.c_void_p),
    ]


class lm_loss_weights(ctypes.Structure):
    _fields_ = [
        ("area", ctypes.c_float),
        ("volume", ctypes.c_float),
        ("sq_norm", ctypes.c_float),
        ("p0", ctypes.c_float * 3),
    ]


class lm_tuning(ctypes.Structure):
    _fields_ = [
        ("v_four_per_wave", ctypes.c_int32),
        ("v_two_per_wave", ctypes.c_int32),
        ("group_nodes", ctypes.c_int64),
    ]


class LatmeshError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {lm_status_string(code)} ({code})")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load liblatmesh.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2405_15197_amd/build.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.lm_plan_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(lm_lattice), P]
    lib.lm_plan_create.restype = ctypes.c_int
    lib.lm_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(lm_options),
                                      ctypes.POINTER(ctypes.c_size_t)]
    lib.lm_workspace_size.restype = ctypes.c_int
    lib.lm_plan_create_in.argtypes = [ctypes.POINTER(P), ctypes.POINTER(lm_lattice), ctypes.POINTER(lm_options), P,
                                      ctypes.c_size_t, P]
    lib.lm_plan_create_in.restype = ctypes.c_int
    lib.lm_plan_create_end_radii.argtypes = [ctypes.POINTER(P), ctypes.POINTER(lm_lattice), P, ctypes.c_float, P,
                                             ctypes.POINTER(ctypes.c_int64), P]
    lib.lm_plan_create_end_radii.restype = ctypes.c_int
    lib.lm_end_radius_gradient.argtypes = [P, P, P]
    lib.lm_end_radius_gradient.restype = ctypes.c_int
    lib.lm_count.argtypes = [P, ctypes.c_int, ctypes.POINTER(lm_totals)]
    lib.lm_count.restype = ctypes.c_int
    lib.lm_fill.argtypes = [P, ctypes.POINTER(lm_outputs)]
    lib.lm_fill.restype = ctypes.c_int
    lib.lm_forward.argtypes = [P, ctypes.c_int, ctypes.POINTER(lm_outputs)]
    lib.lm_forward.restype = ctypes.c_int
    lib.lm_retriangulate.argtypes = [P, ctypes.c_int, ctypes.POINTER(lm_outputs)]
    lib.lm_retriangulate.restype = ctypes.c_int
    lib.lm_read_totals.argtypes = [P, ctypes.POINTER(lm_totals)]
    lib.lm_read_totals.restype = ctypes.c_int
    lib.lm_prepare.argtypes = [P]
    lib.lm_prepare.restype = ctypes.c_int
    lib.lm_set_profiling.argtypes = [P, ctypes.c_int]
    lib.lm_set_profiling.restype = ctypes.c_int
    lib.lm_get_profile.argtypes = [P, P, P, ctypes.c_int]
    lib.lm_get_profile.restype = ctypes.c_int
    lib.lm_set_schedule.argtypes = [P, ctypes.c_int]
    lib.lm_set_schedule.restype = ctypes.c_int
    lib.lm_set_precision.argtypes = [P, ctypes.c_float]
    lib.lm_set_precision.restype = ctypes.c_int
    lib.lm_forward_sink.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, ctypes.c_int64]
    lib.lm_forward_sink.restype = ctypes.c_int
    lib.lm_static_scratch_size.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_size_t)]
    lib.lm_static_scratch_size.restype = ctypes.c_int
    lib.lm_forward_sink_static.argtypes = [ctypes.POINTER(lm_lattice), ctypes.c_int, P, P]
    lib.lm_forward_sink_static.restype = ctypes.c_int
    lib.lm_batched.argtypes = [P, ctypes.c_int64, P, P, ctypes.POINTER(lm_tuning), P]
    lib.lm_batched.restype = ctypes.c_int
    lib.lm_loss.argtypes = [P, ctypes.POINTER(lm_outputs), ctypes.POINTER(lm_loss_weights), P, P]
    lib.lm_loss.restype = ctypes.c_int
    lib.lm_backward.argtypes = [P, P, P, P]
    lib.lm_backward.restype = ctypes.c_int
    lib.lm_write_stl.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_char_p, ctypes.c_int64, ctypes.c_int, P,
                                 ctypes.POINTER(lm_stl_stats)]
    lib.lm_write_stl.restype = ctypes.c_int
    lib.lm_arc_encode.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                                  ctypes.POINTER(lm_arc_codes), ctypes.POINTER(ctypes.c_int64)]
    lib.lm_arc_encode.restype = ctypes.c_int
    lib.lm_arc_decode.argtypes = [P, ctypes.POINTER(lm_arc_codes), P, ctypes.c_int64, ctypes.c_int64, ctypes.c_float,
                                  ctypes.c_float, P, ctypes.c_int64]
    lib.lm_arc_decode.restype = ctypes.c_int
    lib.lm_plan_destroy.argtypes = [P]
    lib.lm_plan_destroy.restype = None
    lib.lm_status_string.argtypes = [ctypes.c_int]
    lib.lm_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


# ---- same-named thin wrappers -------------------------------------------


def lm_status_string(code: int) -> str:
    return load().lm_status_string(int(code)).decode()


def lm_plan_create(lat: lm_lattice, stream: int | None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    rc = load().lm_plan_create(ctypes.byref(h), ctypes.byref(lat), ctypes.c_void_p(stream or 0))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_plan_create")
    return h


def lm_workspace_size(n_nodes: int, n_struts: int, opt: lm_options | None) -> int:
    b = ctypes.c_size_t(0)
    rc = load().lm_workspace_size(int(n_nodes), int(n_struts), ctypes.byref(opt) if opt is not None else None,
                                  ctypes.byref(b))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_workspace_size")
    return int(b.value)


def lm_plan_create_in(lat: lm_lattice, opt: lm_options | None, d_workspace: int, nbytes: int,
                      stream: int | None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    rc = load().lm_plan_create_in(ctypes.byref(h), ctypes.byref(lat), ctypes.byref(opt) if opt is not None else None,
                                  ctypes.c_void_p(d_workspace), int(nbytes), ctypes.c_void_p(stream or 0))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_plan_create_in")
    return h


def lm_plan_create_end_radii(lat: lm_lattice, d_end_radius: int, rel_tol: float, d_radius: int,
                             stream: int | None):
    """(plan, mismatching nodes); raises LatmeshError (code
    LM_ERR_RADIUS_MISMATCH) when end radii at a node differ."""
    h = ctypes.c_void_p()
    nm = ctypes.c_int64(0)
    rc = load().lm_plan_create_end_radii(ctypes.byref(h), ctypes.byref(lat), ctypes.c_void_p(d_end_radius),
                                         float(rel_tol), ctypes.c_void_p(d_radius), ctypes.byref(nm),
                                         ctypes.c_void_p(stream or 0))
    if rc != LM_OK:
        err = LatmeshError(rc, "lm_plan_create_end_radii")
        err.n_mismatch = int(nm.value)
        raise err
    return h, int(nm.value)


def lm_end_radius_gradient(plan, d_grad_radius: int, d_grad_end: int) -> None:
    rc = load().lm_end_radius_gradient(plan, ctypes.c_void_p(d_grad_radius), ctypes.c_void_p(d_grad_end))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_end_radius_gradient")


def lm_count(plan, k: int) -> lm_totals:
    t = lm_totals()
    rc = load().lm_count(plan, int(k), ctypes.byref(t))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_count")
    return t


def lm_fill(plan, out: lm_outputs) -> None:
    rc = load().lm_fill(plan, ctypes.byref(out))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_fill")


def lm_forward(plan, k: int, out: lm_outputs) -> None:
    rc = load().lm_forward(plan, int(k), ctypes.byref(out))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_forward")


def lm_retriangulate(plan, k: int, out: lm_outputs) -> None:
    rc = load().lm_retriangulate(plan, int(k), ctypes.byref(out))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_retriangulate")


def lm_write_stl(d_mesh_xyz: int, n_mesh_vertices: int, d_tri: int, n_triangles: int, path, chunk_bytes: int,
                 flags: int, stream: int | None) -> lm_stl_stats:
    st = lm_stl_stats()
    p = None if path is None else os.fsencode(path)
    rc = load().lm_write_stl(ctypes.c_void_p(d_mesh_xyz), int(n_mesh_vertices), ctypes.c_void_p(d_tri),
                             int(n_triangles), p, int(chunk_bytes), int(flags), ctypes.c_void_p(stream or 0),
                             ctypes.byref(st))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_write_stl")
    return st


def write_stl(mesh_xyz, tri, path, chunk_bytes: int = 64 << 20, fsync: bool = False) -> dict:
    """Binary STL of a device mesh (torch tensors [M, 3] float32 and [T, 3]
    int32 on one GPU) through the library's pipelined writer; path None
    runs the pipeline without a file.  Returns the call's statistics."""
    import torch

    mesh_xyz = mesh_xyz.contiguous()
    tri = tri.contiguous()
    with torch.cuda.device(mesh_xyz.device):
        stream = torch.cuda.current_stream().cuda_stream
        st = lm_write_stl(mesh_xyz.data_ptr(), mesh_xyz.shape[0], tri.data_ptr(), tri.shape[0], path, chunk_bytes,
                          LM_STL_FSYNC if fsync else 0, stream)
    return st.as_dict()


def lm_read_totals(plan) -> lm_totals:
    rc, t = lm_read_totals_rc(plan)
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_read_totals")
    return t


def lm_read_totals_rc(plan):
    """(status, totals): the totals are filled also when the status is
    LM_ERR_CAPACITY, and then give the sizes the skipped writes needed."""
    t = lm_totals()
    rc = load().lm_read_totals(plan, ctypes.byref(t))
    return rc, t


PHASES = ("prepare", "node_fp32", "node_fp64", "sizes", "expand", "bands", "loss", "backward")


def lm_loss(plan, out: lm_outputs, w: lm_loss_weights, d_terms: int, d_dl_dx: int) -> None:
    rc = load().lm_loss(plan, ctypes.byref(out), ctypes.byref(w), ctypes.c_void_p(d_terms), ctypes.c_void_p(d_dl_dx))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_loss")


LM_SINK_WORDS = 8
SINK_FIELDS = ("triangles", "tri_hash", "mesh_vertices", "vert_hash", "sum_x", "sum_y", "sum_z", "bad_nodes")


def lm_forward_sink(plan, k: int, chunk_nodes: int, d_out: int, n_chunks_cap: int) -> None:
    rc = load().lm_forward_sink(plan, int(k), int(chunk_nodes), ctypes.c_void_p(d_out), int(n_chunks_cap))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_forward_sink")


LM_STATIC_SCRATCH_BYTES = 128 << 20


def lm_static_scratch_size(n_nodes: int, n_struts: int, k: int) -> int:
    b = ctypes.c_size_t()
    rc = load().lm_static_scratch_size(int(n_nodes), int(n_struts), int(k), ctypes.byref(b))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_static_scratch_size")
    return int(b.value)


def lm_forward_sink_static(lat: lm_lattice, k: int, d_words: int, stream: int) -> None:
    rc = load().lm_forward_sink_static(ctypes.byref(lat), int(k), ctypes.c_void_p(d_words), ctypes.c_void_p(stream))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_forward_sink_static")


def lm_batched(plan, part_off, part_k, tune, d_out: int) -> None:
    """part_off: int64 numpy [n_parts + 1], part_k: int32 numpy [n_parts]."""
    po = np.ascontiguousarray(part_off, np.int64)
    pk = np.ascontiguousarray(part_k, np.int32)
    rc = load().lm_batched(plan, len(pk), po.ctypes.data_as(ctypes.c_void_p), pk.ctypes.data_as(ctypes.c_void_p),
                           ctypes.byref(tune) if tune is not None else None, ctypes.c_void_p(d_out))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_batched")


def lm_backward(plan, d_dl_dx: int, d_grad_xyz: int, d_grad_radius: int) -> None:
    rc = load().lm_backward(plan, ctypes.c_void_p(d_dl_dx), ctypes.c_void_p(d_grad_xyz),
                            ctypes.c_void_p(d_grad_radius))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_backward")


def lm_prepare(plan) -> None:
    rc = load().lm_prepare(plan)
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_prepare")


def lm_set_profiling(plan, on: bool) -> None:
    rc = load().lm_set_profiling(plan, 1 if on else 0)
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_set_profiling")


def lm_get_profile(plan) -> dict:
    """{phase: (milliseconds summed, calls)} since the last call."""
    ms = np.zeros(len(PHASES), np.float64)
    calls = np.zeros(len(PHASES), np.int64)
    rc = load().lm_get_profile(plan, ms.ctypes.data_as(ctypes.c_void_p), calls.ctypes.data_as(ctypes.c_void_p),
                               len(PHASES))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_get_profile")
    return {p: (float(m), int(c)) for p, m, c in zip(PHASES, ms, calls)}


def lm_set_precision(plan, kappa_max: float) -> None:
    rc = load().lm_set_precision(plan, float(kappa_max))
    if rc != LM_OK:
        raise LatmeshError(rc, "lm_set_precision")


def lm_plan_destroy(plan) -> None:
    load().lm_plan_destroy(plan)


# ---- torch helper ----------------------------------------------------------


@dataclasses.dataclass
class MeshResult:
    totals: dict
    mesh_xyz: object  # torch float32 [M, 3]
    tri: object  # torch int32 [T, 3]
    vert_name: object | None = None  # torch int32 (uint32 bits) [V]
    vert_xyz: object | None = None  # torch float32 [3, V] (node local)
    arc_f32: object | None = None  # torch float32 [11, E]
    arc_u32: object | None = None  # torch int32 (uint32 bits) [3, E]
    node_off: object | None = None  # torch int64 [5, N+1]
    node_status: object | None = None  # torch uint8 [N]
    strut_off: object | None = None  # torch int64 [S+1]


class Mesher:
    """Owns device copies of a lattice and one plan.  ``lat`` is any object
    with x, y, z, radius (float32) and strut_a, strut_b (int32) arrays.
    ``options`` (an lm_options): the plan takes all of its device memory from
    one buffer allocated here (lm_plan_create_in) instead of allocating it
    itself.  ``end_radius`` ([S, 2] per-strut end radii): the node radii are
    derived from them (lm_plan_create_end_radii, tolerance ``rel_tol``)."""

    def __init__(self, lat, device: str = "cuda:0", kappa_max: float | None = None, options=None,
                 end_radius=None, rel_tol: float = 0.0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("latmesh needs a GPU (torch.cuda.is_available() is False)")
        load()
        self.torch = torch
        self.device = torch.device(device)
        def f(a, dt):
            if isinstance(a, torch.Tensor):  # already a tensor (e.g. generated on the device)
                return a.to(device=self.device, dtype=dt).contiguous()
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(self.device)

        self.x = f(lat.x, torch.float32)
        self.y = f(lat.y, torch.float32)
        self.z = f(lat.z, torch.float32)
        self.r = f(lat.radius, torch.float32)
        self.sa = f(lat.strut_a, torch.int32)
        self.sb = f(lat.strut_b, torch.int32)
        self.n_nodes = int(self.x.shape[0])
        self.n_struts = int(self.sa.shape[0])
        self._lat = lm_lattice(
            self.n_nodes,
            self.n_struts,
            self.x.data_ptr(),
            self.y.data_ptr(),
            self.z.data_ptr(),
            self.r.data_ptr(),
            self.sa.data_ptr(),
            self.sb.data_ptr(),
        )
        self.workspace = None
        self.end_radius = None
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream().cuda_stream
            if end_radius is not None:
                self.end_radius = f(end_radius, torch.float32).reshape(-1, 2).contiguous()
                self.plan, _ = lm_plan_create_end_radii(self._lat, self.end_radius.data_ptr(), rel_tol,
                                                        self.r.data_ptr(), self.stream)
            elif options is not None:
                nb = lm_workspace_size(self.n_nodes, self.n_struts, options)
                # 256-byte aligned (the caching allocator aligns blocks to 512)
                self.workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=self.device)
                self.plan = lm_plan_create_in(self._lat, options, self.workspace.data_ptr(), nb, self.stream)
            else:
                self.plan = lm_plan_create(self._lat, self.stream)
        if kappa_max is not None:
            lm_set_precision(self.plan, kappa_max)
        self.totals = None
        self.k = 0

    def count(self, k: int) -> dict:
        self.totals = lm_count(self.plan, k).as_dict()
        self.k = k
        return self.totals

    def alloc(self, totals: dict | None = None, meta: bool = True) -> MeshResult:
        torch = self.torch
        t = totals or self.totals
        dev = self.device
        r = MeshResult(
            totals=dict(t),
            mesh_xyz=torch.empty((max(t["n_mesh_vertices"], 1), 3), dtype=torch.float32, device=dev),
            tri=torch.empty((max(t["n_triangles"], 1), 3), dtype=torch.int32, device=dev),
        )
        if meta:
            r.vert_name = torch.empty(max(t["n_vertices"], 1), dtype=torch.int32, device=dev)
            r.vert_xyz = torch.empty((3, max(t["n_vertices"], 1)), dtype=torch.float32, device=dev)
            r.arc_f32 = torch.empty((11, max(t["n_arcs"], 1)), dtype=torch.float32, device=dev)
            r.arc_u32 = torch.empty((3, max(t["n_arcs"], 1)), dtype=torch.int32, device=dev)
        r.node_off = torch.empty((5, self.n_nodes + 1), dtype=torch.int64, device=dev)
        r.node_status = torch.empty(max(self.n_nodes, 1), dtype=torch.uint8, device=dev)
        r.strut_off = torch.empty(self.n_struts + 1, dtype=torch.int64, device=dev)
        return r

    def outputs(self, r: MeshResult) -> lm_outputs:
        p = lambda x: x.data_ptr() if x is not None else None  # noqa: E731
        return lm_outputs(
            p(r.mesh_xyz),
            p(r.tri),
            r.mesh_xyz.shape[0],
            r.tri.shape[0],
            p(r.vert_name),
            p(r.vert_xyz),
            r.vert_name.shape[0] if r.vert_name is not None else 0,
            p(r.arc_f32),
            p(r.arc_u32),
            r.arc_f32.shape[1] if r.arc_f32 is not None else 0,
            p(r.node_off),
            p(r.node_status),
            p(r.strut_off),
        )

    def fill(self, r: MeshResult) -> MeshResult:
        lm_fill(self.plan, self.outputs(r))
        return r

    def run(self, k: int, meta: bool = True) -> MeshResult:
        """count + allocate + fill; returns device tensors trimmed to size."""
        t = self.count(k)
        r = self.fill(self.alloc(t, meta=meta))
        self.torch.cuda.synchronize(self.device)
        err = lm_read_totals(self.plan)  # raises on device-side errors
        return self._trim(r, err.as_dict(), meta)

    def retriangulate(self, k: int, meta: bool = True, r: MeshResult | None = None) -> MeshResult:
        """Subdivide the meta-mesh of the last count / run / forward again at
        k without re-solving the nodes.  Writes into ``r`` when given and
        large enough, else into buffers sized from the totals (a second call
        when the first guess was too small); returns trimmed tensors."""
        if r is None:
            # the last call's totals (none yet: lm_retriangulate refuses)
            base = lm_read_totals_rc(self.plan)[1].as_dict() if self.k else dict.fromkeys(_TOTAL_FIELDS, 0)
            f = max(1.0, k / max(self.k, 1)) * 1.05
            t = {key: int(v * f) + 64 for key, v in base.items()}
            r = self.alloc(t, meta=meta)
        for attempt in range(2):
            lm_retriangulate(self.plan, k, self.outputs(r))
            rc, tt = lm_read_totals_rc(self.plan)
            if rc == LM_OK:
                break
            if rc != LM_ERR_CAPACITY or attempt == 1:
                raise LatmeshError(rc, "lm_retriangulate")
            r = self.alloc(tt.as_dict(), meta=meta)
        return self._trim(r, tt.as_dict(), meta)

    def write_stl(self, r: MeshResult, path, chunk_bytes: int = 64 << 20, fsync: bool = False) -> dict:
        """Binary STL of the mesh in ``r`` (trimmed to its totals)."""
        t = r.totals
        return write_stl(r.mesh_xyz[: t["n_mesh_vertices"]], r.tri[: t["n_triangles"]], path, chunk_bytes, fsync)

    def set_schedule(self, thread_centric: bool) -> None:
        """FP32 node pass: wave-centric (default) or the thread-centric
        ablation (one lane per node, scratch in global memory)."""
        rc = load().lm_set_schedule(self.plan, 1 if thread_centric else 0)
        if rc != LM_OK:
            raise LatmeshError(rc, "lm_set_schedule")

    def radius_range(self):
        """(smallest, largest) node radius of the lattice."""
        return float(self.r.min().item()), float(self.r.max().item())

    def encode_arcs(self, r: MeshResult, r_min=None, r_max=None, cap_fallback=None) -> dict:
        """128-bit codes of the meta-mesh arcs in ``r`` (a MeshResult with
        meta-mesh arrays); returns device tensors ``codes`` [E, 4] int32
        (bit patterns), ``mask`` [(E + 31) // 32], ``fallback`` [F, 11] and
        the host int ``n_fallback``."""
        torch = self.torch
        lo, hi = self.radius_range()
        r_min = lo if r_min is None else r_min
        r_max = hi if r_max is None else r_max
        E = r.arc_f32.shape[1]
        cap_fb = max(E // 16, 64) if cap_fallback is None else cap_fallback
        dev = self.device
        codes = torch.empty((max(E, 1), 4), dtype=torch.int32, device=dev)
        mask = torch.empty(max((E + 31) // 32, 1), dtype=torch.int32, device=dev)
        fb = torch.empty((max(cap_fb, 1), 11), dtype=torch.float32, device=dev)
        c = lm_arc_codes(codes.data_ptr(), mask.data_ptr(), fb.data_ptr(), codes.shape[0], cap_fb)
        nf = ctypes.c_int64(0)
        ld = r.arc_f32.stride(0)
        rc = load().lm_arc_encode(self.plan, ctypes.c_void_p(r.arc_f32.data_ptr()),
                                  ctypes.c_void_p(r.arc_u32.data_ptr()), E, ld, r_min, r_max, ctypes.byref(c),
                                  ctypes.byref(nf))
        if rc != LM_OK:
            raise LatmeshError(rc, "lm_arc_encode")
        return {"codes": codes[:E], "mask": mask, "fallback": fb[: nf.value], "n_fallback": nf.value,
                "cap_fallback": cap_fb, "r_min": r_min, "r_max": r_max, "_fb_full": fb}

    def decode_arcs(self, enc: dict, r: MeshResult):
        """Arcs [11, E] float32 (the fields of arc_f32) from encode_arcs' output."""
        torch = self.torch
        E = enc["codes"].shape[0]
        out = torch.empty((11, max(E, 1)), dtype=torch.float32, device=self.device)
        c = lm_arc_codes(enc["codes"].data_ptr(), enc["mask"].data_ptr(), enc["_fb_full"].data_ptr(),
                         max(E, 1), enc["cap_fallback"])
        rc = load().lm_arc_decode(self.plan, ctypes.byref(c), ctypes.c_void_p(r.arc_u32.data_ptr()), E,
                                  r.arc_u32.stride(0), enc["r_min"], enc["r_max"], ctypes.c_void_p(out.data_ptr()),
                                  out.stride(0))
        if rc != LM_OK:
            raise LatmeshError(rc, "lm_arc_decode")
        return out[:, :E]

    def _trim(self, r: MeshResult, t: dict, meta: bool) -> MeshResult:
        r.totals = t
        r.mesh_xyz = r.mesh_xyz[: t["n_mesh_vertices"]]
        r.tri = r.tri[: t["n_triangles"]]
        if meta:
            r.vert_name = r.vert_name[: t["n_vertices"]]
            r.vert_xyz = r.vert_xyz[:, : t["n_vertices"]]
            r.arc_f32 = r.arc_f32[:, : t["n_arcs"]]
            r.arc_u32 = r.arc_u32[:, : t["n_arcs"]]
        r.node_status = r.node_status[: self.n_nodes]
        return r

    def forward(self, k: int, r: MeshResult, check: bool = False) -> None:
        """lm_forward into ``r``; with check, synchronise and raise when the
        pass skipped writes (buffers or records too small) or its mesh sizes
        differ from r.totals (a different topology than the buffers hold)."""
        lm_forward(self.plan, k, self.outputs(r))
        self.k = k
        if check:
            rc, t = lm_read_totals_rc(self.plan)
            if rc != LM_OK:
                raise LatmeshError(rc, "lm_forward")
            t = t.as_dict()
            for key in ("n_mesh_vertices", "n_triangles"):
                if t[key] != r.totals[key]:
                    raise LatmeshError(LM_ERR_STATE, f"lm_forward: {key} {t[key]} differs from the buffers' "
                                                     f"{r.totals[key]} (topology changed)")

    def loss(self, r: MeshResult, weights=(1.0, 0.0, 0.0), p0=(0.0, 0.0, 0.0)):
        """Loss terms (area, volume about p0, sum |v|^2) of the mesh in ``r``
        and dL/dx of the weighted loss; returns (terms float64 [3], dl_dx
        float32 [M, 3]) as device tensors."""
        torch = self.torch
        terms = torch.zeros(3, dtype=torch.float64, device=self.device)
        dl = torch.empty((r.mesh_xyz.shape[0], 3), dtype=torch.float32, device=self.device)
        w = lm_loss_weights(float(weights[0]), float(weights[1]), float(weights[2]),
                            (ctypes.c_float * 3)(*[float(x) for x in p0]))
        lm_loss(self.plan, self.outputs(r), w, terms.data_ptr(), dl.data_ptr())
        return terms, dl

    def end_radius_grad(self, grad_radius):
        """[S, 2] gradient with respect to the end radii of a plan made from
        end radii, from a gradient with respect to the node radii."""
        torch = self.torch
        g = torch.empty((self.n_struts, 2), dtype=torch.float32, device=self.device)
        lm_end_radius_gradient(self.plan, grad_radius.contiguous().data_ptr(), g.data_ptr())
        return g

    def backward(self, dl_dx):
        """Gradient with respect to node centres [N, 3] and radii [N] of a
        loss whose gradient with respect to the last mesh is ``dl_dx``."""
        torch = self.torch
        dl_dx = dl_dx.contiguous()
        gx = torch.empty((self.n_nodes, 3), dtype=torch.float32, device=self.device)
        gr = torch.empty(self.n_nodes, dtype=torch.float32, device=self.device)
        lm_backward(self.plan, dl_dx.data_ptr(), gx.data_ptr(), gr.data_ptr())
        return gx, gr

    def sink(self, k: int, chunk_nodes: int):
        """Chunked meshing reduced to per-chunk counts and hashes; returns a
        uint64 numpy array [chunks, LM_SINK_WORDS] (see SINK_FIELDS)."""
        torch = self.torch
        nch = max((self.n_nodes + chunk_nodes - 1) // chunk_nodes, 1)
        out = torch.zeros((nch, LM_SINK_WORDS), dtype=torch.int64, device=self.device)
        lm_forward_sink(self.plan, k, chunk_nodes, out.data_ptr(), nch)
        self.torch.cuda.synchronize(self.device)
        return out.cpu().numpy().view(np.uint64)

    def batched(self, part_off, part_k, tune=None):
        """Per-part sink words (uint64 numpy [parts, LM_SINK_WORDS]) of the
        parts [part_off[p], part_off[p+1]) at resolutions part_k."""
        torch = self.torch
        out = torch.zeros((len(part_k), LM_SINK_WORDS), dtype=torch.int64, device=self.device)
        lm_batched(self.plan, part_off, part_k, tune, out.data_ptr())
        torch.cuda.synchronize(self.device)
        return out.cpu().numpy().view(np.uint64)

    def set_inputs(self, xyz, radius) -> None:
        """Copy new node centres [N, 3] and radii [N] (device tensors) into the
        plan's lattice and redo its preparation (same struts)."""
        self.x.copy_(xyz[:, 0])
        self.y.copy_(xyz[:, 1])
        self.z.copy_(xyz[:, 2])
        self.r.copy_(radius)
        lm_prepare(self.plan)

    def close(self):
        if getattr(self, "plan", None) is not None:
            lm_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mesh_function():
    """torch.autograd.Function: (xyz [N, 3], radius [N]) -> mesh vertices
    [M, 3] of ``mesher`` at resolution k; its backward is lm_backward (the
    adjoint at the forward pass's topology).  Usage:
    ``verts = mesh_function().apply(xyz, radius, mesher, k, result)`` with
    ``result`` a MeshResult sized by an earlier ``mesher.count(k)``."""
    import torch

    class MeshFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, xyz, radius, mesher, k, result):
            mesher.set_inputs(xyz.detach(), radius.detach())
            # raises if the new inputs changed the topology the buffers were
            # sized for (then the adjoint would not match the mesh)
            mesher.forward(k, result, check=True)
            ctx.mesher = mesher
            return result.mesh_xyz.clone()

        @staticmethod
        def backward(ctx, grad_verts):
            gx, gr = ctx.mesher.backward(grad_verts)
            return gx, gr, None, None, None

    return MeshFn
