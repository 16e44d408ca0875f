"""Thread-centric ablation of the FP32 node pass (one lane per node, scratch
in global memory): against the FP64 oracle element by element (the parity
bar of tests/parity.py), and bit-identical to the wave-centric pass (the
same node code), including nodes handed to FP64 and nodes of more than 16
struts."""

import numpy as np
import pytest

import latgen
from parity import compare, result_np

pytestmark = pytest.mark.gpu

CASES = [
    ("cfg2_bcc5", lambda: latgen.config(2, scale=5), 16),
    ("cfg4_octet3", lambda: latgen.config(4, scale=3), 12),
    ("cubic_cones", lambda: latgen.cubic(5, radius=("uniform", 0.05, 0.15), jitter=0.04, seed=5), 8),
    ("cfg3_bcc5_unjittered", lambda: latgen.config(3, scale=5), 12),
    # random k-NN: valences above 16 (the multi-wave class), many invalid nodes
    ("knn5_12", lambda: latgen.knn(5, 12, radius=0.12, seed=3), 9),
    ("knn5_18", lambda: latgen.knn(5, 18, radius=("uniform", 0.04, 0.12), seed=518), 12),
]


@pytest.mark.parametrize("name,make,k", CASES, ids=[c[0] for c in CASES])
def test_thread_schedule_matches_wave(name, make, k):
    from paper_2405_15197_amd import Mesher

    lat = make()
    out = []
    for thread in (False, True):
        M = Mesher(lat)
        try:
            M.set_schedule(thread)
            out.append(result_np(M.run(k)))
        finally:
            M.close()
    a, b = out
    print(f"schedule {name}: {a['totals']}", flush=True)
    ta = {key: v for key, v in a["totals"].items() if key != "n_record_bytes"}
    tb = {key: v for key, v in b["totals"].items() if key != "n_record_bytes"}
    assert ta == tb
    for key in ("status", "node_off", "strut_off", "vert_name", "vert_xyz", "arc_u32", "arc_f32", "tri", "mesh"):
        assert np.array_equal(a[key], b[key]), key
    st = compare(lat, k, G=b)
    print(f"  thread schedule against the oracle: {st}", flush=True)
