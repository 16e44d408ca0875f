"""Nodes of more than 16 struts: the multi-wave class (a block of several
waves per node sharing its LDS, Sec. 4.3.3 "several warps for a heavy
workload") against the FP64 oracle, through the C ABI.

Random k-NN lattices (the batched workload's fourth family, k up to 20,
symmetrised: valences up to about 40) have most of their nodes in that class.
The comparison is the same element-by-element one as for the one-wave
classes (tests/parity.py): status, counts, names, arcs, mesh vertices and
triangles of every node whose oracle margins are above the comparison
thresholds.
"""

import numpy as np
import pytest

import latgen
import oracle
from parity import above_margin, compare, gpu_result

pytestmark = pytest.mark.gpu

RAD = ("uniform", 0.04, 0.12)
KNN = [
    ("knn6_20_k16", lambda: latgen.knn(6, 20, radius=RAD, seed=620), 16),
    ("knn8_16_k12", lambda: latgen.knn(8, 16, radius=RAD, seed=816), 12),
    ("knn5_12_k9", lambda: latgen.knn(5, 12, radius=RAD, seed=512), 9),
    ("knn7_18_k8", lambda: latgen.knn(7, 18, radius=RAD, seed=718), 8),
    ("knn4_18_k32", lambda: latgen.knn(4, 18, radius=RAD, seed=418), 32),
]


def _line(msg):
    print(msg, flush=True)


def _valence(lat):
    return np.bincount(np.concatenate([lat.strut_a, lat.strut_b]), minlength=lat.n_nodes)


@pytest.mark.parametrize("name,make,k", KNN, ids=[c[0] for c in KNN])
def test_knn_parity(name, make, k):
    lat = make()
    v = _valence(lat)
    _line(f"knn {name}: {lat.n_nodes} nodes, {lat.n_struts} struts, valence <= {v.max()}, k={k}")
    R = oracle.run(lat, k)
    G = gpu_result(lat, k)
    st = compare(lat, k, R=R, G=G)
    stable_big = int((((R.status == 0) & above_margin(R, k)) & (v > 16)).sum())
    _line(f"  {st}, stable nodes above 16 struts: {stable_big}")
    assert stable_big > 0
    # every node the oracle meshes is meshed (those below the margin too)
    meshed = G["status"] == 0
    assert (meshed[R.status == 0]).mean() >= 0.98
    assert st["stable"] >= 0.9 * int((R.status == 0).sum())


@pytest.mark.parametrize("nstrut", [17, 24, 33, 40, 48, 56, 64])
def test_star_valence(nstrut):
    """A centre node with nstrut thin struts in quasi-random directions (a
    Fibonacci sphere, jittered): meshed by the multi-wave class, equal to
    the oracle."""
    i = np.arange(nstrut) + 0.5
    phi = np.arccos(1 - 2 * i / nstrut)
    th = np.pi * (1 + 5 ** 0.5) * i + 0.1 * np.sin(7 * i)
    d = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    lat = latgen.star(d, radius=0.05)
    st = compare(lat, 12, tau=1e-6)
    _line(f"star {nstrut}: {st}")
    assert st["stable"] == lat.n_nodes


@pytest.mark.parametrize("nstrut", [20, 32, 33, 48])
def test_star_valence_all_fp64(nstrut):
    """kappa_max = 0: the star's node meshed by the FP64 pass, on two waves
    up to 32 struts and on four above; equal to the oracle."""
    i = np.arange(nstrut) + 0.5
    phi = np.arccos(1 - 2 * i / nstrut)
    th = np.pi * (1 + 5 ** 0.5) * i + 0.1 * np.sin(7 * i)
    d = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    lat = latgen.star(d, radius=0.05)
    st = compare(lat, 12, tau=1e-8, geom_tol=1e-6, kappa_max=0.0)
    _line(f"star {nstrut}, FP64: {st}")
    assert st["fp64_nodes"] == lat.n_nodes
    assert st["stable"] == lat.n_nodes


def test_valence_beyond_limit_is_flagged():
    i = np.arange(72) + 0.5
    phi = np.arccos(1 - 2 * i / 72)
    th = np.pi * (1 + 5 ** 0.5) * i
    d = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    lat = latgen.star(d, radius=0.01)
    G = gpu_result(lat, 8, meta=False)
    assert G["status"][0] & 32  # LM_NODE_VALENCE
    assert (G["status"][1:] == 0).all()


def test_knn_all_fp64():
    """kappa_max = 0: every node, the multi-wave class included, meshed by the
    FP64 pass; combinatorics equal to the oracle above margin 1e-8."""
    lat = latgen.knn(5, 17, radius=RAD, seed=517)
    st = compare(lat, 12, tau=1e-8, geom_tol=1e-6, kappa_max=0.0)
    _line(f"  {st}")
    assert st["fp64_nodes"] == lat.n_nodes


def test_knn_retriangulate_equals_forward():
    """Re-subdivision solves multi-wave nodes again (their records are not
    re-read), so it gives the bits of lm_forward at the new k."""
    import torch

    from paper_2405_15197_amd import Mesher
    from parity import result_np

    lat = latgen.knn(6, 19, radius=RAD, seed=619)
    M = Mesher(lat)
    try:
        M.run(16)
        a = result_np(M.retriangulate(9))
    finally:
        M.close()
    b = gpu_result(lat, 9)
    torch.cuda.synchronize()
    for key in ("status", "node_off", "strut_off", "vert_name", "vert_xyz", "arc_u32", "arc_f32", "tri", "mesh"):
        assert np.array_equal(a[key], b[key]), key


def _fib_dirs(n, wobble=0.1):
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = np.pi * (1 + 5 ** 0.5) * i + wobble * np.sin(7 * i)
    return np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


@pytest.mark.parametrize("nstrut", [20, 31])
def test_high_valence_gradient_matches_oracle(nstrut):
    """The adjoint of a node of more than 16 struts (its own kernel
    instantiation, over the multi-wave class's queue) against the oracle's
    FP64 central differences: every parameter of the centre node and of
    three of its neighbours, conical struts (seeded end-node radii)."""
    import torch

    from paper_2405_15197_amd import Mesher

    rng = np.random.default_rng(nstrut)
    d = _fib_dirs(nstrut) * rng.uniform(0.8, 1.2, size=(nstrut, 1))
    radii = np.concatenate([[0.08], rng.uniform(0.04, 0.07, size=nstrut)])
    xyz = np.concatenate([np.zeros((1, 3)), d])
    lat = latgen.lattice_from_arrays(xyz, radii, [(0, i + 1) for i in range(nstrut)])
    k = 12
    R = oracle.run(lat, k)
    assert (R.status == 0).all()
    params = [(n, c) for n in (0, 1, 5, nstrut) for c in range(4)]
    G, ok = oracle.fd_gradient(lat, k, params, weights=[(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)])
    assert ok.all()
    M = Mesher(lat)
    try:
        r = M.run(k, meta=False)
        for wi, w in enumerate(((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))):
            terms, dl = M.loss(r, w)
            gx, gr = M.backward(dl)
            torch.cuda.synchronize()
            gx, gr = gx.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64)
            g_gpu = np.array([gx[n, c] if c < 3 else gr[n] for n, c in params])
            g_orc = G[:, wi]
            tol = 1e-3 * np.abs(g_orc) + 1e-4 * np.abs(g_orc).max()
            err = np.abs(g_gpu - g_orc)
            assert (err <= tol).all(), (wi, (err / tol).max(), params[int(np.argmax(err / tol))])
    finally:
        M.close()
