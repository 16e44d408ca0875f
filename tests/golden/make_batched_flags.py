"""Writes batched512_oracle_flags.json: for every part of the 512-part
batched workload (latgen.parts(512, seed=1)), the number of nodes the FP64
oracle leaves without a mesh (any non-zero status: valence, topology,
degenerate input), the part's node count and its resolution k.  Uses only
the input generator and the oracle; about 2.5 hours on 6 host threads.

    python tests/golden/make_batched_flags.py [threads]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import latgen  # noqa: E402
from oracle import _load, _p  # noqa: E402


def unmeshed(lat, k, threads):
    """Nodes of ``lat`` the oracle leaves without a mesh at resolution k (the
    status column only; the mesh itself is not copied out)."""
    lib = _load()
    a = [np.ascontiguousarray(v, np.float32) for v in (lat.x, lat.y, lat.z, lat.radius)]
    sa = np.ascontiguousarray(lat.strut_a, np.int32)
    sb = np.ascontiguousarray(lat.strut_b, np.int32)
    h = lib.orc_run(len(a[0]), len(sa), *(_p(v) for v in a), _p(sa), _p(sb), int(k), int(threads))
    cnt = np.zeros((len(a[0]), 8), np.int32)
    mg = np.zeros(len(a[0]), np.float64)
    lib.orc_nodes(h, _p(cnt), _p(mg))
    lib.orc_free(h)
    return int((cnt[:, 0] != 0).sum())


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    t0 = time.time()
    per = []
    for i, (lat, k) in enumerate(latgen.parts(512, seed=1, workers=threads)):
        per.append([unmeshed(lat, k, threads), lat.n_nodes, int(k)])
        if i % 32 == 0:
            print(i, lat.name, f"{time.time() - t0:.0f} s", flush=True)
    out = {
        "recipe": "latgen.parts(512, seed=1); per part [oracle nodes without a mesh, nodes, k]",
        "flagged": sum(p[0] for p in per),
        "per_part": per,
    }
    json.dump(out, open(os.path.join(HERE, "batched512_oracle_flags.json"), "w"))
    print("flagged", out["flagged"], "of", sum(p[1] for p in per))


if __name__ == "__main__":
    main()
