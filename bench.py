"""Benchmark: meta-meshing + triangulation of the BCC 64^3 lattice on one GPU.

One step is the whole path on one synthetic lattice already resident in HBM:
validation and adjacency (lm_prepare), per-node meta-meshing and counts,
prefix sums, the fill pass (meta-mesh, mesh vertices, hole fans) and the
strut bands (lm_forward), into preallocated device buffers.

Prints one JSON line (see README of the benchmark contract in the design
notes): struts/s as the value, triangles/s beside it, the roofline entry of
the dominant kernel measured with HIP events inside the library, and the
FP64 CPU oracle timed on the same lattice (by default the whole of it).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

# HBM bytes per launch of the node kernel, from FETCH_SIZE / WRITE_SIZE
# counter runs scaled by a plain copy's readings (factors 2.0 / 1.0), keyed
# by the kernel's sources and build flags they were taken on; a changed
# kernel reports null.
MEASURED_TRAFFIC = {
    "7722bb1d9b107fad": {"bytes": 2_354_991_016, "summary": "profiles/k_node32_bcc64_k16_hbm_counters.md"},
}
# wave64 VALU instructions per node pass (SQ_INSTS_VALU summed over its
# launches) from the same counter runs, keyed the same way
MEASURED_VALU = {
    "7722bb1d9b107fad": {"insts": 1_353_826_481, "summary": "profiles/k_node32_bcc64_k16_hbm_counters.md"},
}
# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per
# SIMD every 4 cycles (16 lanes wide; packed FP32 is not used)
VALU_PEAK_GINSTS = 256 * 4 * 2.4 / 4


def node_source_key():
    import hashlib

    h = hashlib.sha256()
    for f in ("csrc/node.hip", "csrc/common.h", "csrc/geom.h", "build.py"):
        with open(os.path.join(ROOT, "paper_2405_15197_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(lat, t):
    """Bytes the method must move once per step: read the lattice, write the
    meta-mesh (16 B per vertex: name + xyz; 56 B per arc: o, a, b, t1, t2,
    labels, end vertices, node) and the indexed mesh (12 B per vertex, 12 B
    per triangle)."""
    read = 16 * lat.n_nodes + 8 * lat.n_struts
    meta = 16 * t["n_vertices"] + 56 * t["n_arcs"]
    mesh = 12 * t["n_mesh_vertices"] + 12 * t["n_triangles"]
    return read, meta, mesh


def node_kernel_bytes(lat, t):
    """Algorithmic bytes of the per-node meta-meshing kernel: it reads the
    lattice (16 B per node, 8 B per strut) and produces the meta-mesh (16 B
    per meta-vertex, 56 B per arc)."""
    read = 16 * lat.n_nodes + 8 * lat.n_struts
    return read + 16 * t["n_vertices"] + 56 * t["n_arcs"]


def host_cpu():
    """CPU model and logical CPU count of the host (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(scale: int, k: int, threads: int):
    import latgen
    import oracle

    oracle.build(force=False)
    lat = latgen.config(2, scale=scale, seed=1)
    t0 = time.perf_counter()
    R = oracle.run(lat, k, threads=threads)
    dt = time.perf_counter() - t0
    excl = excluded_fractions(R, lat, k)
    # the billion-strut family (no jitter) on a 24^3 sample
    lat3 = latgen.config(3, scale=24, seed=1)
    excl3 = excluded_fractions(oracle.run(lat3, 12, threads=threads), lat3, 12)
    return {
        "value": lat.n_struts / dt,
        "unit": "struts/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": host_cpu()[0],
        "host_logical_cpus": host_cpu()[1],
        "sample": f"BCC {scale}^3 cells ({lat.n_nodes} nodes, {lat.n_struts} struts), k={k}, same seeded "
        f"distributions as the GPU workload, meta-mesh + triangulation, FP64 C oracle, {dt:.1f} s wall",
        "triangles_per_s": len(R.tris) / dt,
        # nodes and struts the parity tests leave out of the element-wise
        # comparison (oracle margins below the per-kind thresholds)
        "excluded": {"bcc64_k16": excl, "billion_family_bcc24_k12": excl3},
    }


def excluded_fractions(R, lat, k):
    """Shares of the nodes and struts below the parity tests' comparison
    thresholds (the tests' own per-kind margins)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import STRUT_TAU, above_margin

    above = above_margin(R, k)
    sa, sb = lat.strut_a.astype(np.int64), lat.strut_b.astype(np.int64)
    ok = (R.strut_status == 0) & above[sa] & above[sb]
    return {"nodes": float(1.0 - above.mean()),
            "struts": float(1.0 - (ok & (R.strut_margin >= STRUT_TAU)).mean())}


def copy_probe(mib: int):
    """A plain device-to-device copy of known size, for scaling the profiler's
    FETCH_SIZE / WRITE_SIZE readings to bytes."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": 4 * n, "launches": 5}), flush=True)


def adjoint_bench(steps: int, warmup: int, k: int = 16):
    """Forward, and forward + loss + adjoint, on the octet-truss 32^3 lattice
    (FCC sites, 12 nearest neighbours, radii U[0.04, 0.10], jitter 0.03):
    the loss is Area + Vol + 1e-3 sum|v|^2 over the mesh."""
    import torch

    import latgen
    from paper_2405_15197_amd.latmesh import (Mesher, lm_backward, lm_forward, lm_loss, lm_loss_weights,
                                              lm_prepare, lm_read_totals)
    import ctypes

    lat = latgen.config(4, seed=1)
    M = Mesher(lat)
    t = M.count(k)
    r = M.alloc(t, meta=False)
    out = M.outputs(r)
    terms = torch.zeros(3, dtype=torch.float64, device="cuda")
    dl = torch.empty((r.mesh_xyz.shape[0], 3), dtype=torch.float32, device="cuda")
    gx = torch.empty((lat.n_nodes, 3), dtype=torch.float32, device="cuda")
    gr = torch.empty(lat.n_nodes, dtype=torch.float32, device="cuda")
    w = lm_loss_weights(1.0, 1.0, 1e-3, (ctypes.c_float * 3)(0.0, 0.0, 0.0))

    def fwd():
        lm_prepare(M.plan)
        lm_forward(M.plan, k, out)

    def fwd_bwd():
        fwd()
        lm_loss(M.plan, out, w, terms.data_ptr(), dl.data_ptr())
        lm_backward(M.plan, dl.data_ptr(), gx.data_ptr(), gr.data_ptr())

    res = {}
    for name, fn in (("fwd", fwd), ("fwd_bwd", fwd_bwd)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        res[name] = a.elapsed_time(b) / steps
    lm_read_totals(M.plan)
    M.close()
    return {
        "workload": f"octet 32^3 cells, {lat.n_nodes} nodes, {lat.n_struts} struts, radii U[0.04,0.10], jitter 0.03, "
        f"k={k}, loss Area + Vol + 1e-3 sum|v|^2",
        "fwd_ms": res["fwd"],
        "fwd_bwd_ms": res["fwd_bwd"],
        "fwd_bwd_per_s": 1e3 / res["fwd_bwd"],
        "ratio": res["fwd_bwd"] / res["fwd"],
    }


def retri_bench(M, k0: int, ks, steps: int, warmup: int):
    """Re-subdivision of the k0 meta-mesh at other resolutions against a
    forward pass at those resolutions, on the plan's lattice."""
    import torch

    from paper_2405_15197_amd.latmesh import (lm_forward, lm_get_profile, lm_read_totals, lm_retriangulate,
                                              lm_set_profiling)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    def phases(fn):
        lm_get_profile(M.plan)
        lm_set_profiling(M.plan, True)
        fn()
        prof = lm_get_profile(M.plan)
        lm_set_profiling(M.plan, False)
        return {p: round(v[0], 4) for p, v in prof.items() if v[1]}

    out = {"k0": k0}
    for k in ks:
        M.count(k0)
        r = M.retriangulate(k, meta=True)  # sizes the buffers
        o = M.outputs(r)
        f_ms = timed(lambda: lm_forward(M.plan, k, o))
        f_ph = phases(lambda: lm_forward(M.plan, k, o))
        lm_forward(M.plan, k0, M.outputs(M.alloc(M.count(k0), meta=True)))
        r_ms = timed(lambda: lm_retriangulate(M.plan, k, o))
        r_ph = phases(lambda: lm_retriangulate(M.plan, k, o))
        lm_read_totals(M.plan)
        out[f"k{k}"] = {"forward_ms": f_ms, "retriangulate_ms": r_ms, "speedup": f_ms / r_ms,
                        "triangles": r.totals["n_triangles"], "forward_phase_ms": f_ph,
                        "retriangulate_phase_ms": r_ph}
    return out


def stl_bench(scale: int = 64, k: int = 16, path_dir: str | None = None):
    """Binary STL of the BCC mesh through the pipelined writer: without a
    file (encode + PCIe copy only), to a file with fsync at several chunk
    sizes, and the disk and the PCIe copy alone for the same bytes."""
    import tempfile

    import torch

    import latgen
    from paper_2405_15197_amd.latmesh import Mesher

    lat = latgen.config(2, scale=scale, seed=1)
    M = Mesher(lat)
    r = M.run(k, meta=False)
    t = r.totals
    nbytes = 84 + 50 * t["n_triangles"]
    d = path_dir or os.environ.get("TMPDIR") or tempfile.gettempdir()
    path = os.path.join(d, f"latmesh_bench_{os.getpid()}.stl")
    out = {"workload": f"BCC {scale}^3 cells, k={k}: {t['n_triangles']} triangles, {nbytes} bytes", "bytes": nbytes,
           "dir": d}
    try:
        M.write_stl(r, None)  # warm-up: allocations, first launches
        st = M.write_stl(r, None)
        out["no_file"] = {"GB_per_s": nbytes / st["seconds"] / 1e9, **st}
        for mib in (16, 64, 256):
            st = M.write_stl(r, path, chunk_bytes=mib << 20, fsync=True)
            out[f"file_fsync_{mib}MiB"] = {"GB_per_s": nbytes / st["seconds"] / 1e9, **st}
            os.remove(path)
        # the disk alone: the same bytes from one host buffer, fsync at the end
        buf = np.zeros(64 << 20, np.uint8)
        t0 = time.perf_counter()
        fd = os.open(path, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o644)
        left = nbytes
        while left > 0:
            left -= os.write(fd, memoryview(buf)[: min(left, buf.size)])
        os.fsync(fd)
        os.close(fd)
        out["disk_only_GB_per_s"] = nbytes / (time.perf_counter() - t0) / 1e9
        os.remove(path)
        # the same from pinned host memory (what the pipeline writes from)
        pbuf = torch.zeros(64 << 20, dtype=torch.uint8, pin_memory=True).numpy()
        t0 = time.perf_counter()
        fd = os.open(path, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o644)
        left = nbytes
        while left > 0:
            left -= os.write(fd, memoryview(pbuf)[: min(left, pbuf.size)])
        os.fsync(fd)
        os.close(fd)
        out["disk_only_pinned_GB_per_s"] = nbytes / (time.perf_counter() - t0) / 1e9
        os.remove(path)
        # the PCIe copy alone: device to pinned host, 64 MiB pieces
        dev = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
        host = torch.empty(64 << 20, dtype=torch.uint8, pin_memory=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        left = nbytes
        while left > 0:
            n = min(left, dev.numel())
            host[:n].copy_(dev[:n], non_blocking=True)
            left -= n
        torch.cuda.synchronize()
        out["d2h_only_GB_per_s"] = nbytes / (time.perf_counter() - t0) / 1e9
    finally:
        if os.path.exists(path):
            os.remove(path)
        M.close()
    return out


def codec_bench(scale: int = 64, k: int = 16, steps: int = 10):
    """Arc codec on the benchmark meta-mesh: encode and decode times, bytes
    against the FP32 arcs (44 B) and the node records' arc fields (64 B),
    fallback share, and the Eq. 5 error on a sample of arcs."""
    import torch

    import latgen
    from paper_2405_15197_amd.latmesh import Mesher

    lat = latgen.config(2, scale=scale, seed=1)
    M = Mesher(lat)
    try:
        r = M.run(k, meta=True)
        E = r.arc_f32.shape[1]
        enc = M.encode_arcs(r)
        dec = M.decode_arcs(enc, r)

        def timed(fn):
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                fn()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / steps

        enc_ms = timed(lambda: M.encode_arcs(r))  # includes its synchronisation
        dec_ms = timed(lambda: M.decode_arcs(enc, r))
        rng = np.random.default_rng(0)
        sel = np.sort(rng.choice(E, size=min(E, 200000), replace=False))
        arcs = r.arc_f32.cpu().numpy().T[sel].astype(np.float64)
        dd = dec.cpu().numpy().T[sel].astype(np.float64)
        mask = enc["mask"].cpu().numpy().view(np.uint32)
        fb = ((mask[sel >> 5] >> (sel & 31)) & 1).astype(bool)
        # distance between arc and decoded arc at equal t, 17 samples per arc
        a0, a1 = arcs[~fb], dd[~fb]
        t = a0[:, 9:10] + (a0[:, 10:11] - a0[:, 9:10]) * np.linspace(0.0, 1.0, 17)[None, :]
        st, ct = np.sin(t)[:, :, None], np.cos(t)[:, :, None]
        pa = a0[:, None, 0:3] + a0[:, None, 3:6] * st + a0[:, None, 6:9] * ct
        pb = a1[:, None, 0:3] + a1[:, None, 3:6] * st + a1[:, None, 6:9] * ct
        err = np.linalg.norm(pa - pb, axis=2).max(axis=1)
        # Eq. 5 with n = 12, m = 15
        q1, q2 = 2.0 ** (2 * 12 + 2), 32.0 * np.pi ** 2 / 2.0 ** (2 * 15 + 2)
        eq5 = float(np.sqrt(17.0 / q1 + q2) + np.sqrt(1.0 / q1 + q2))
        nf = enc["n_fallback"]
        code_bytes = 16 * E + 44 * nf + 4 * ((E + 31) // 32)
        return {
            "workload": f"BCC {scale}^3 cells, k={k}: {E} meta-mesh arcs",
            "arcs": E,
            "fallback": nf,
            "fallback_share": nf / E,
            "bytes_fp32_arcs": 44 * E,
            "bytes_codes": code_bytes,
            "ratio_vs_fp32_arcs": 44 * E / code_bytes,
            "encode_ms": enc_ms,
            "decode_ms": dec_ms,
            "encode_arcs_per_s": E / (enc_ms * 1e-3),
            "decode_arcs_per_s": E / (dec_ms * 1e-3),
            "max_error_over_r_max_sampled": float(err.max() / enc["r_max"]),
            "eq5_bound": eq5,
        }
    finally:
        M.close()


def ablation_bench(scale: int = 64, k: int = 16, steps: int = 3):
    """The FP32 node pass (lm_count's meta-meshing) wave-centric against the
    thread-centric ablation (one lane per node, scratch in global memory),
    device time from the library's events."""
    import torch

    import latgen
    from paper_2405_15197_amd.latmesh import Mesher, lm_get_profile, lm_set_profiling

    lat = latgen.config(2, scale=scale, seed=1)
    M = Mesher(lat)
    out = {"workload": f"BCC {scale}^3 cells, {lat.n_nodes} nodes, k={k}: FP32 node pass"}
    try:
        for name, thread in (("wave_centric", False), ("thread_centric", True)):
            M.set_schedule(thread)
            M.count(k)  # warm-up (and the thread pass's scratch)
            torch.cuda.synchronize()
            lm_get_profile(M.plan)
            lm_set_profiling(M.plan, True)
            for _ in range(steps):
                M.count(k)
            prof = lm_get_profile(M.plan)
            lm_set_profiling(M.plan, False)
            out[name + "_ms"] = prof["node_fp32"][0] / max(prof["node_fp32"][1], 1)
        out["speedup_wave_over_thread"] = out["thread_centric_ms"] / out["wave_centric_ms"]
    finally:
        M.close()
    return out


def billion_bench(k: int = 12, chunk_nodes: int = 1 << 23, scale: int = 512):
    """The BCC 512^3 lattice (269,223,425 nodes, 1,073,741,824 struts; radii
    0.08 (1 + U[-0.1, 0.1]), no jitter), generated on the device, meshed in
    sink mode: per chunk of node ids, counts and order-independent hashes
    instead of a stored mesh.  One pass, timed with HIP events."""
    import torch

    import latgen.device
    from paper_2405_15197_amd.latmesh import SINK_FIELDS, Mesher

    print(f"[bench] generating BCC {scale}^3 on the device", file=sys.stderr, flush=True)
    lat = latgen.device.config(3, scale=scale)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M = Mesher(lat)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    print(f"[bench] plan ready in {t_plan:.1f} s; sink pass", file=sys.stderr, flush=True)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    words = M.sink(k, chunk_nodes)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    with np.errstate(over="ignore"):
        tot = words.sum(axis=0, dtype=np.uint64)
    M.close()
    tot = {f: int(v) for f, v in zip(SINK_FIELDS, tot)}
    return {
        "metric": "struts meta-meshed/s (and triangles emitted/s) at resolution k",
        "value": lat.n_struts / (ms * 1e-3),
        "unit": "struts/s",
        "n_gpus": 1,
        "ms_per_pass": ms,
        "triangles_per_s": tot["triangles"] / (ms * 1e-3),
        "config": {
            "workload": f"BCC {scale}^3 cells, {lat.n_nodes} nodes, {lat.n_struts} struts, radii 0.08(1+U[-0.1,0.1]), "
            f"no jitter, k={k}, sink mode (per-chunk counts + hashes), chunks of {chunk_nodes} node ids",
        },
        "plan_s": t_plan,
        "sink_totals": tot,
        "chunks": int(words.shape[0]),
    }


def make_parts(n_parts: int = 512, n_max: int = 64, seed: int = 1):
    """The batched workload's parts, built on the host in worker processes
    (before this process touches the GPU); returns (parts, seconds)."""
    import latgen

    t0 = time.perf_counter()
    print(f"[bench] generating {n_parts} parts", file=sys.stderr, flush=True)
    parts = latgen.parts(n_parts, seed=seed, n_max=n_max, workers=min(16, os.cpu_count() or 1))
    return parts, time.perf_counter() - t0


def batched_bench(n_parts: int = 512, n_max: int = 64, seed: int = 1, pre=None):
    """512 lattice parts (cubic, BCC, octet or random k-NN, 4..64 cells per
    side, radii U[0.04, 0.12], resolutions 8/16/32) meshed in sink mode:
    batched (one plan, autotuned wave mapping and group size, one node pass
    per group of parts) against the parts one after another (a plan each,
    its own launches).  Host-side generation and plan creation are not
    timed; both sides time preparation (adjacency) + meshing."""
    import torch

    import latgen
    from paper_2405_15197_amd.autotune import tune
    from paper_2405_15197_amd.latmesh import Mesher, lm_get_profile, lm_prepare, lm_set_profiling

    parts, t_gen = pre if pre is not None else make_parts(n_parts, n_max, seed)
    t0 = time.perf_counter()
    lat, off = latgen.union([p[0] for p in parts])
    ks = np.array([p[1] for p in parts], np.int32)
    t_gen += time.perf_counter() - t0
    print(f"[bench] {lat.n_nodes} nodes, {lat.n_struts} struts ({t_gen:.0f} s); autotuning", file=sys.stderr,
          flush=True)
    best, table = tune(parts, latgen.union, sample=32)
    M = Mesher(lat)
    M.batched(off, ks, best)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lm_prepare(M.plan)
    words = M.batched(off, ks, best)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    # the same call again with the library's phase timers on (not the timed run)
    lm_get_profile(M.plan)
    lm_set_profiling(M.plan, True)
    M.batched(off, ks, best)
    prof = lm_get_profile(M.plan)
    lm_set_profiling(M.plan, False)
    phase_ms = {p: round(v[0], 3) for p, v in prof.items() if v[1]}
    M.close()
    print(f"[bench] batched {t_batched:.2f} s; sequential per-part baseline", file=sys.stderr, flush=True)
    t_seq = 0.0
    seq_words = []
    for i, (pl, k) in enumerate(parts):
        Mp = Mesher(pl)
        try:
            Mp.sink(int(k), max(pl.n_nodes, 1))  # warm-up (allocations)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lm_prepare(Mp.plan)
            seq_words.append(Mp.sink(int(k), max(pl.n_nodes, 1))[0])
            torch.cuda.synchronize()
            t_seq += time.perf_counter() - t0
        finally:
            Mp.close()
        if i % 64 == 63:
            print(f"[bench]   {i + 1} parts", file=sys.stderr, flush=True)
    same = bool(np.array_equal(np.stack(seq_words), words))
    with np.errstate(over="ignore"):
        tot = words.sum(axis=0, dtype=np.uint64)
    return {
        "metric": "struts meta-meshed/s (and triangles emitted/s) at resolution k",
        "value": lat.n_struts / t_batched,
        "unit": "struts/s",
        "n_gpus": 1,
        "config": {"workload": f"{n_parts} parts (cubic/BCC/octet/k-NN, 4..{n_max} cells, k in 8/16/32), "
                   f"{lat.n_nodes} nodes, {lat.n_struts} struts, sink mode per part"},
        "batched_s": t_batched,
        "sequential_s": t_seq,
        "speedup_vs_sequential": t_seq / t_batched,
        "identical_to_sequential": same,
        "tuning": {"v_four_per_wave": best.v_four_per_wave, "v_two_per_wave": best.v_two_per_wave,
                   "group_nodes": best.group_nodes},
        "tuning_table_ms": {f"{a},{b},{c}": v for (a, b, c), v in table.items()},
        "triangles": int(tot[0]),
        "triangles_per_s": int(tot[0]) / t_batched,
        "nodes_without_mesh": int(tot[7]),
        "phase_ms": phase_ms,
        "generation_s": t_gen,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--scale", type=int, default=64, help="BCC cells per side (64 = the benchmarked lattice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-scale", type=int, default=64, help="BCC cells per side of the oracle's lattice")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward + adjoint leg (octet 32^3)")
    ap.add_argument("--adjoint", action="store_true", help="only the forward + adjoint leg (octet 32^3)")
    ap.add_argument("--no-retri", action="store_true", help="skip the re-subdivision leg")
    ap.add_argument("--stl", action="store_true", help="only the binary STL writer on the benchmark mesh")
    ap.add_argument("--codec", action="store_true", help="only the arc codec on the benchmark meta-mesh")
    ap.add_argument("--ablation", action="store_true",
                    help="only the node pass, wave-centric against the thread-centric ablation")
    ap.add_argument("--billion", action="store_true",
                    help="only the BCC 512^3 lattice in sink mode (generated on the device), one pass")
    ap.add_argument("--billion-scale", type=int, default=512)
    ap.add_argument("--batched", action="store_true", help="only the 512-part batch (sink mode), batched vs sequential")
    ap.add_argument("--no-billion", action="store_true", help="skip the billion-strut sink leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-part batched leg")
    ap.add_argument("--batched-parts", type=int, default=512)
    ap.add_argument("--batched-nmax", type=int, default=64)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB a few times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.billion:
        print(json.dumps(billion_bench(scale=args.billion_scale)), flush=True)
        return
    if args.batched:
        print(json.dumps(batched_bench(args.batched_parts, args.batched_nmax)), flush=True)
        return
    if args.stl:
        print(json.dumps(stl_bench(args.scale, args.k)), flush=True)
        return
    if args.codec:
        print(json.dumps(codec_bench(args.scale, args.k)), flush=True)
        return
    if args.ablation:
        print(json.dumps(ablation_bench(args.scale, args.k)), flush=True)
        return
    if args.adjoint:
        print(json.dumps(adjoint_bench(args.steps, args.warmup)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU design is in the "
              "design notes and not built", file=sys.stderr)
        sys.exit(2)
    # the batched leg's parts are built first, in worker processes forked
    # before anything here initialises the GPU
    pre_parts = None if args.no_batched else make_parts(args.batched_parts, args.batched_nmax)

    import torch

    import latgen
    from paper_2405_15197_amd.latmesh import Mesher, lm_get_profile, lm_prepare, lm_read_totals, lm_set_profiling

    print(f"[bench] building BCC {args.scale}^3 lattice", file=sys.stderr, flush=True)
    lat = latgen.config(2, scale=args.scale, seed=1)
    M = Mesher(lat)
    t = M.count(args.k)
    buf = M.alloc(t, meta=True)
    out = M.outputs(buf)
    from paper_2405_15197_amd.latmesh import lm_forward

    def step():
        lm_prepare(M.plan)
        lm_forward(M.plan, args.k, out)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lm_read_totals(M.plan)  # raises on device-side errors
    lm_get_profile(M.plan)  # drop anything recorded so far
    lm_set_profiling(M.plan, True)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    start.record()
    for _ in range(args.steps):
        step()
    end.record()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(end)
    prof = lm_get_profile(M.plan)
    lm_set_profiling(M.plan, False)
    tot = lm_read_totals(M.plan).as_dict()
    assert tot == t or all(tot[key] == t[key] for key in t if key != "n_fp64_nodes"), (tot, t)
    ms = ms_total / args.steps
    struts_s = lat.n_struts / (ms * 1e-3)
    tris_s = tot["n_triangles"] / (ms * 1e-3)
    read, meta, mesh = algorithmic_bytes(lat, tot)
    phase_ms = {p: (v[0] / max(v[1], 1)) for p, v in prof.items()}
    dominant = max(phase_ms, key=phase_ms.get)
    fb = node_kernel_bytes(lat, tot)
    kern_ms = phase_ms["node_fp32"]
    achieved = fb / (kern_ms * 1e-3) / 1e9
    mt = MEASURED_TRAFFIC.get(node_source_key())
    traffic = mt["bytes"] if mt else None
    mv = MEASURED_VALU.get(node_source_key())
    valu = None
    if mv:
        gi = mv["insts"] / (kern_ms * 1e-3) / 1e9
        valu = {"kernel": "k_node32 (per-node meta-meshing, FP32)", "bound": "alu", "achieved": gi,
                "peak": VALU_PEAK_GINSTS, "unit": "G wave64 VALU instructions/s", "frac": gi / VALU_PEAK_GINSTS,
                "insts_per_launch": mv["insts"]}
    res = {
        "metric": "struts meta-meshed/s (and triangles emitted/s) at resolution k",
        "value": struts_s,
        "unit": "struts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 for ill-conditioned nodes)",
        "data": "synthetic (seeded BCC lattice)",
        "config": {
            "workload": f"BCC {args.scale}^3 cells, {lat.n_nodes} nodes, {lat.n_struts} struts, node radii "
            f"U[0.05,0.12], jitter 0.05, k={args.k}, stored meta-mesh + indexed mesh",
            "k": args.k,
            "nodes": lat.n_nodes,
            "struts": lat.n_struts,
        },
        "triangles_per_s": tris_s,
        "triangles": tot["n_triangles"],
        "mesh_vertices": tot["n_mesh_vertices"],
        "fp64_nodes": tot["n_fp64_nodes"],
        "path_algorithmic_bytes": read + meta + mesh,
        "path_hbm_frac": (read + meta + mesh) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "phase_ms": phase_ms,
        "dominant_phase": dominant,
        "roofline": {
            "kernel": "k_node32 (per-node meta-meshing, FP32)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": fb,
            "ms_per_launch": kern_ms,
        },
        # the same kernel against the vector-ALU issue rate, which is what
        # bounds it (null when its source differs from the one counted)
        "alu_roofline": valu,
    }
    if not args.no_retri:
        print("[bench] re-subdivision of the k=16 meta-mesh", file=sys.stderr, flush=True)
        res["retriangulate"] = retri_bench(M, args.k, (8, 32), args.steps, args.warmup)
    M.close()
    if not args.no_adjoint:
        print("[bench] forward + adjoint on octet 32^3", file=sys.stderr, flush=True)
        res["fwd_bwd"] = adjoint_bench(args.steps, args.warmup)
    if not args.no_billion:
        print("[bench] billion-strut lattice in sink mode", file=sys.stderr, flush=True)
        res["billion"] = billion_bench(scale=args.billion_scale)
    if not args.no_batched:
        print("[bench] 512-part batch", file=sys.stderr, flush=True)
        res["batched"] = batched_bench(args.batched_parts, args.batched_nmax, pre=pre_parts)
        pre_parts = None
    if not args.no_cpu_baseline:
        # one GPU's share of the host is 16 hardware threads, whatever
        # os.cpu_count() reports for the whole machine
        threads = min(16, os.cpu_count() or 1)
        print(f"[bench] CPU oracle baseline on {threads} threads", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(args.cpu_scale, args.k, threads)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
