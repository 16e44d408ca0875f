"""Device-side generation of the seeded BCC lattices (bit-identical to
``latgen.bcc``), for lattices too large to build on the host.  Input
generation only: ``gen.hip`` holds none of the meshing arithmetic."""

from __future__ import annotations

import ctypes
import os
import subprocess
import types

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.hip")
_LIB = os.path.join(_HERE, "libgen.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.hip for gfx950 (no floating-point contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-ffp-contract=off", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", _SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on gen.hip:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError(f"{_LIB} is missing: run latgen.device.build() (or __graft_entry__.build())")
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.lg_bcc.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_uint64, ctypes.c_double] + [P] * 7
        lib.lg_bcc.restype = ctypes.c_int
        _lib = lib
    return _lib


def bcc(n, radius=0.1, jitter=0.0, seed=1, cell=1.0, order="grid", device="cuda:0"):
    """latgen.bcc(n, radius, jitter, seed, cell, order) generated on the GPU; returns
    a namespace of device tensors x, y, z, radius (float32), strut_a,
    strut_b (int32)."""
    import torch

    m = n + 1
    N, S = m**3 + n**3, 8 * n**3
    if isinstance(radius, (int, float)):
        kind, a, b = 0, float(radius), 0.0
    elif radius[0] == "uniform":
        kind, a, b = 1, float(radius[1]), float(radius[2] - radius[1])
    elif radius[0] == "rel":
        kind, a, b = 2, float(radius[1]), float(radius[2])
    else:
        raise ValueError(f"unknown radius spec {radius!r}")
    if order not in ("grid", "layer"):
        raise ValueError(f"unknown node order {order!r}")
    dev = torch.device(device)
    f = lambda k, dt: torch.empty(k, dtype=dt, device=dev)  # noqa: E731
    x, y, z, r = (f(N, torch.float32) for _ in range(4))
    sa, sb = f(S, torch.int32), f(S, torch.int32)
    with torch.cuda.device(dev):
        st = torch.cuda.current_stream().cuda_stream
        rc = _load().lg_bcc(int(n), 0 if order == "grid" else 1, kind, a, b, float(jitter), int(seed), float(cell),
                            x.data_ptr(), y.data_ptr(), z.data_ptr(), r.data_ptr(), sa.data_ptr(), sb.data_ptr(),
                            ctypes.c_void_p(st))
    if rc != 0:
        raise RuntimeError(f"lg_bcc failed with HIP error {rc}")
    return types.SimpleNamespace(x=x, y=y, z=z, radius=r, strut_a=sa, strut_b=sb, n_nodes=N, n_struts=S,
                                 name=f"bcc{n}" + ("" if order == "grid" else "L"))


def config(i: int, seed: int = 1, scale: int | None = None, device="cuda:0"):
    """The BCC workloads of latgen.config (2 and 3) on the device."""
    if i == 2:
        return bcc(scale or 64, radius=("uniform", 0.05, 0.12), jitter=0.05, seed=seed, device=device)
    if i == 3:
        return bcc(scale or 512, radius=("rel", 0.08, 0.1), jitter=0.0, seed=seed, order="layer", device=device)
    raise ValueError(f"no device generator for config {i}")
