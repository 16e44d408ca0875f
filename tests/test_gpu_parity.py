"""GPU path against the FP64 oracle (through the C ABI)."""

import numpy as np
import pytest

import latgen
import oracle
from parity import STRUT_TAU, above_margin, check_closed, compare, gpu_result, sub_lattice

pytestmark = pytest.mark.gpu


def _line(msg):
    print(msg, flush=True)


WORKED = {
    "ljoint": lambda: latgen.star([[1, 0, 0], [0, 1, 0]], radius=0.1),
    "corner": lambda: latgen.star([[1, 0, 0], [0, 1, 0], [0, 0, 1]], radius=0.1),
    "capsule_cone": lambda: latgen.lattice_from_arrays([(0, 0, 0), (1, 0.3, 0.2)], [0.1, 0.06], [(0, 1)]),
    "capsule_big_end": lambda: latgen.lattice_from_arrays([(0, 0, 0), (1, 0, 0)], [0.12, 0.05], [(0, 1)]),
    "star5": lambda: latgen.star([[1, 0.1, 0], [0, 1, 0.2], [-1, 0.1, 0.3], [0.2, -1, 0.1], [0.1, 0.2, 1]],
                                 radius=0.12),
    "obtuse_cones": lambda: latgen.lattice_from_arrays(
        [(0, 0, 0), (1, 0, 0), (np.cos(1.9), np.sin(1.9), 0.1)], [0.1, 0.07, 0.14], [(0, 1), (0, 2)]),
}


@pytest.mark.parametrize("name", sorted(WORKED))
@pytest.mark.parametrize("k", [5, 9, 16])
def test_worked_cases(name, k):
    lat = WORKED[name]()
    _line(f"worked {name} k={k}")
    # symmetric inputs: every node is compared; struts whose end loops share
    # phi values only approximately (margin < 1e-6) are skipped, except
    # between two whole tangency circles, where both sides use the same
    # sub-parameters and the ties are exact
    st = compare(lat, k, tau=0.0, strut_tau=-1.0 if name.startswith("capsule") else 1e-6)
    assert st["stable"] == lat.n_nodes


CONFIGS = [
    ("cfg1_cubic6", lambda: latgen.config(1), 8),
    ("cfg1_cubic6_k13", lambda: latgen.config(1), 13),
    ("cfg2_bcc5", lambda: latgen.config(2, scale=5), 16),
    ("cfg2_bcc9_seed2", lambda: latgen.config(2, scale=9, seed=2), 16),
    ("cfg2_bcc7_k7", lambda: latgen.config(2, scale=7, seed=3), 7),
    ("cfg4_octet3", lambda: latgen.config(4, scale=3), 16),
    ("cubic_cones", lambda: latgen.cubic(5, radius=("uniform", 0.05, 0.15), jitter=0.04, seed=5), 12),
    ("bcc_cyl", lambda: latgen.bcc(4, radius=0.1, jitter=0.05, seed=9), 11),
    # unjittered: exactly opposite struts and seams at exactly half turns
    ("cfg3_bcc6_unjittered", lambda: latgen.config(3, scale=6), 12),
    ("cfg3_bcc5_jitter", lambda: latgen.bcc(5, radius=("rel", 0.08, 0.1), jitter=0.01, seed=4), 12),
]


@pytest.mark.parametrize("name,make,k", CONFIGS, ids=[c[0] for c in CONFIGS])
def test_config_parity(name, make, k):
    lat = make()
    _line(f"config {name}: {lat.n_nodes} nodes {lat.n_struts} struts k={k}")
    R = oracle.run(lat, k)
    G = gpu_result(lat, k)
    st = compare(lat, k, R=R, G=G)
    chi, vol = check_closed(G, lat)
    _line(f"  {st}; closed, chi {chi}, volume {vol:.4g}")
    # small lattices: a handful of nodes below the margins
    assert st["stable"] >= 0.98 * lat.n_nodes


BUDGET = [
    # the benchmark lattice's family (BCC, radii U[0.05, 0.12], jitter 0.05)
    ("cfg2_bcc16", lambda: latgen.config(2, scale=16, seed=5), 16, 0.003),
    # the billion-strut lattice's family (BCC, radii 0.08 (1 +- 0.1), no jitter)
    ("cfg3_bcc14", lambda: latgen.config(3, scale=14, seed=2), 12, 0.02),
]


@pytest.mark.parametrize("name,make,k,budget", BUDGET, ids=[c[0] for c in BUDGET])
def test_exclusion_budget(name, make, k, budget):
    """Nodes below the comparison margins stay within the budget (0.3 % on
    the benchmark family, 2 % on the unjittered billion-strut family), every
    other node and strut equals the oracle, and the whole GPU mesh is closed
    and oriented (so the excluded nodes are checked for a valid surface)."""
    lat = make()
    R = oracle.run(lat, k)
    G = gpu_result(lat, k)
    st = compare(lat, k, R=R, G=G)
    chi, vol = check_closed(G, lat)
    excl = 1.0 - st["stable"] / lat.n_nodes
    strut_excl = 1.0 - (st["stable_struts"] + st["tied_struts"]) / lat.n_struts
    _line(f"  {st}; excluded nodes {excl:.4%}, struts compared by vertex set only {st['tied_struts']}, "
          f"not compared {strut_excl:.4%}; closed, chi {chi}")
    assert excl <= budget


def test_full_config2_sampled():
    """BCC 64^3 (536,769 nodes, 2,097,152 struts) at k = 16 as benchmarked:
    the whole mesh is watertight with Euler characteristic 2N - 2S, and
    sampled nodes (and the struts between sampled nodes) match the oracle,
    which sees only the stars of the samples."""
    import torch

    lat = latgen.config(2)
    k = 16
    _line("full config 2: GPU run")
    G = gpu_result(lat, k, meta=True)
    t = G["totals"]
    _line(f"  totals {t}")
    # near-degenerate nodes that FP32 cannot resolve are redone in FP64
    assert t["n_bad_nodes"] == 0 and t["n_skipped_struts"] == 0
    # watertight + oriented, on the GPU
    tri = torch.as_tensor(G["tri"], device="cuda")
    M = int(t["n_mesh_vertices"])
    e0 = torch.cat([tri[:, 0], tri[:, 1], tri[:, 2]])
    e1 = torch.cat([tri[:, 1], tri[:, 2], tri[:, 0]])
    key = torch.sort(e0 * M + e1).values
    assert bool((key[1:] != key[:-1]).all()), "a directed edge is used twice"
    rkey = e1 * M + e0
    pos = torch.searchsorted(key, rkey).clamp(max=key.numel() - 1)
    assert bool((key[pos] == rkey).all()), "an edge has no opposite twin"
    und = int(key.numel()) // 2
    used = int(torch.unique(tri).numel())
    assert used == M
    assert M - und + tri.shape[0] == 2 * lat.n_nodes - 2 * lat.n_struts
    del tri, e0, e1, key, rkey, pos
    # sampled nodes: stars re-meshed by the oracle
    rng = np.random.default_rng(5)
    centres = np.sort(rng.choice(lat.n_nodes, size=1500, replace=False))
    sub, nmap, keep_s = sub_lattice(lat, centres)
    _line(f"  oracle on {sub.n_nodes} nodes around {len(centres)} samples")
    R = oracle.run(sub, k)
    above = above_margin(R, k)
    off = G["node_off"]
    ok = 0
    for n in centres:
        m = nmap[n]
        if R.status[m] != 0 or not above[m]:
            continue
        ok += 1
        assert G["status"][n] == 0
        gv = slice(off[0][n], off[0][n + 1])
        ov = slice(R.vert_off[m], R.vert_off[m + 1])
        assert np.array_equal(G["vert_name"][gv], R.vert_name[ov])
        assert np.abs(G["vert_xyz"][gv] - R.vert_w[ov]).max() <= 1e-5 * lat.radius[n]
        ga = slice(off[1][n], off[1][n + 1])
        oa = slice(R.arc_off[m], R.arc_off[m + 1])
        assert np.array_equal(G["arc_u32"][ga][:, 1] & 0xFFFF, R.arc_int[oa][:, 2])
        assert np.array_equal(G["arc_u32"][ga][:, 1] >> 16, R.arc_int[oa][:, 3])
        gmv = G["mesh"][off[3][n]:off[3][n + 1]]
        omv = R.mesh[R.mesh_off[m]:R.mesh_off[m + 1]]
        assert gmv.shape == omv.shape
        tol = 1e-5 * lat.radius[n] + np.spacing(np.float32(np.abs(omv).max()))
        assert np.abs(gmv - omv).max() <= tol
    assert ok >= 0.995 * len(centres)
    # struts whose both ends are samples
    sa, sb = lat.strut_a.astype(np.int64), lat.strut_b.astype(np.int64)
    both = np.zeros(lat.n_nodes, bool)
    both[centres] = True
    checked = 0
    sub_index = {s: i for i, s in enumerate(keep_s)}
    for s in np.nonzero(both[sa] & both[sb])[0]:
        i = sub_index[s]
        a, b = nmap[sa[s]], nmap[sb[s]]
        if R.status[a] or R.status[b] or not (above[a] and above[b]) or R.strut_margin[i] < STRUT_TAU:
            continue
        gt = G["tri"][G["strut_off"][s]:G["strut_off"][s + 1]]
        ot = R.tris[R.band_off[i]:R.band_off[i + 1]]
        assert gt.shape == ot.shape
        gn = np.searchsorted(off[3], gt, side="right") - 1
        on = np.searchsorted(R.mesh_off, ot, side="right") - 1
        inv = np.full(sub.n_nodes, -1)
        inv[nmap[nmap >= 0]] = np.nonzero(nmap >= 0)[0]
        assert np.array_equal(gn, inv[on])
        assert np.array_equal(gt - off[3][gn], ot - R.mesh_off[on])
        checked += 1
    _line(f"  sampled nodes ok {ok}, struts checked {checked}")


@pytest.mark.parametrize("name,make,k", [CONFIGS[0], CONFIGS[5], CONFIGS[2]], ids=["cfg1", "octet3", "bcc5"])
def test_all_nodes_fp64(name, make, k):
    """kappa_max = 0 meshes every node in FP64: combinatorics identical to the
    oracle on every node with margin >= 1e-8, positions to FP32 output
    rounding (1e-6 rho beyond one ulp)."""
    lat = make()
    st = compare(lat, k, tau=1e-8, geom_tol=1e-6, kappa_max=0.0)
    _line(f"  {st}")
    assert st["fp64_nodes"] == lat.n_nodes
    assert st["stable"] >= 0.999 * lat.n_nodes


def test_forward_matches_count_fill_and_repeats():
    """lm_forward into preallocated buffers (the benchmarked call) writes the
    same bits as lm_count + lm_fill, on every repeat and after a k change."""
    import torch

    from paper_2405_15197_amd import Mesher

    lat = latgen.config(2, scale=6)
    M = Mesher(lat)
    try:
        ref = M.run(16)
        ref_mesh, ref_tri = ref.mesh_xyz.clone(), ref.tri.clone()
        buf = M.alloc(ref.totals)
        for k in (16, 9, 16, 16):
            M.forward(k, buf)
            torch.cuda.synchronize()
            from paper_2405_15197_amd.latmesh import lm_read_totals

            t = lm_read_totals(M.plan).as_dict()
            if k == 16:
                assert t == ref.totals
                assert torch.equal(buf.mesh_xyz[: t["n_mesh_vertices"]], ref_mesh)
                assert torch.equal(buf.tri[: t["n_triangles"]], ref_tri)
    finally:
        M.close()


def test_edge_cases():
    import torch

    from paper_2405_15197_amd import Mesher
    from paper_2405_15197_amd.latmesh import LM_ERR_BAD_LATTICE, LM_ERR_CAPACITY, LatmeshError

    # empty lattice
    empty = latgen.lattice_from_arrays(np.zeros((0, 3)), np.zeros(0), np.zeros((0, 2)))
    M = Mesher(empty)
    t = M.count(8)
    assert t["n_triangles"] == 0 and t["n_mesh_vertices"] == 0
    M.close()
    # isolated nodes and a self loop
    lat = latgen.lattice_from_arrays([(0, 0, 0), (1, 0, 0), (5, 5, 5)], [0.1, 0.1, 0.1], [(0, 1), (2, 2)])
    M = Mesher(lat)
    r = M.run(8)
    st = r.node_status.cpu().numpy()
    assert st[0] == 0 and st[1] == 0 and st[2] & 1
    R = oracle.run(lat, 8)
    assert (R.status != 0).tolist() == (st != 0).tolist()
    M.close()
    # duplicate strut
    lat = latgen.lattice_from_arrays([(0, 0, 0), (1, 0, 0)], [0.1, 0.1], [(0, 1), (1, 0)])
    M = Mesher(lat)
    r = M.run(8)
    assert (r.node_status.cpu().numpy() & 64).all()
    M.close()
    # |r_a - r_b| >= L
    lat = latgen.lattice_from_arrays([(0, 0, 0), (0.1, 0, 0)], [0.3, 0.1], [(0, 1)])
    M = Mesher(lat)
    r = M.run(8)
    assert (r.node_status.cpu().numpy() & 1).all()
    M.close()
    # valence beyond the build limit (64 struts)
    d = np.random.default_rng(1).normal(size=(72, 3))
    lat = latgen.star(d, radius=0.005)
    M = Mesher(lat)
    r = M.run(8)
    assert r.node_status.cpu().numpy()[0] & 32
    M.close()
    # strut index out of range
    bad = latgen.lattice_from_arrays([(0, 0, 0), (1, 0, 0)], [0.1, 0.1], [(0, 1)])
    bad.strut_b = np.array([7], np.int32)
    with pytest.raises(LatmeshError) as ei:
        Mesher(bad)
    assert ei.value.code == LM_ERR_BAD_LATTICE
    # buffers too small
    lat = latgen.config(1)
    M = Mesher(lat)
    t = M.count(8)
    small = dict(t)
    small["n_triangles"] -= 1
    r = M.alloc(small, meta=False)
    with pytest.raises(LatmeshError) as ei:
        M.fill(r)
    assert ei.value.code == LM_ERR_CAPACITY
    M.close()
    torch.cuda.synchronize()


def test_determinism():
    lat = latgen.config(2, scale=5, seed=7)
    a = gpu_result(lat, 16)
    b = gpu_result(lat, 16)
    for key in ("mesh", "tri", "vert_name", "arc_f32"):
        assert np.array_equal(a[key], b[key])
