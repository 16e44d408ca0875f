"""Pins of the oracle's gradient (the reference for the adjoint).

The oracle differentiates the mesh loss L = w_area Area + w_vol Vol +
w_sq sum|v|^2 with respect to node centres and radii at fixed topology, by
central differences in FP64 (``oracle.fd_gradient``).  These tests pin it to
exact properties of the triangulated surface, independent of any
implementation:

* Euler's theorem: scaling every centre and radius by s scales the mesh by
  s (same topology), so Area and sum|v|^2 are homogeneous of degree 2 and
  the volume about the origin of degree 3: sum_j theta_j dL/dtheta_j = d L.
* Translation: moving every centre by u moves every mesh vertex by u, so
  the area and the volume of the closed surface do not change (the
  x-derivatives over all nodes sum to zero), while sum|v|^2 changes by
  2 u . sum v.
"""

import numpy as np
import pytest

import latgen
import oracle


W3 = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]


@pytest.fixture(scope="module")
def small():
    lat = latgen.config(4, scale=2, seed=2)
    R = oracle.run(lat, 12)
    assert (R.status == 0).all()
    params = [(n, c) for n in range(lat.n_nodes) for c in range(4)]
    g, ok = oracle.fd_gradient(lat, 12, params, weights=W3)
    assert ok.all()
    return lat, R, params, g


def _theta(lat, params):
    f = (lat.x, lat.y, lat.z, lat.radius)
    return np.array([float(f[c][n]) for n, c in params])


@pytest.mark.parametrize("weights,degree", [((1, 0, 0), 2), ((0, 1, 0), 3), ((0, 0, 1), 2)])
def test_euler_homogeneity(small, weights, degree):
    lat, R, params, G = small
    g = G[:, W3.index(weights)]
    L = (weights[0] * oracle.mesh_area(R.mesh, R.tris)
         + weights[1] * float(np.einsum("ij,ij->i", R.mesh[R.tris[:, 0]],
                                        np.cross(R.mesh[R.tris[:, 1]], R.mesh[R.tris[:, 2]])).sum() / 6)
         + weights[2] * oracle.mesh_sq(R.mesh))
    lhs = float(np.dot(_theta(lat, params), g))
    assert abs(lhs - degree * L) <= 1e-6 * abs(L), (lhs, degree * L)


@pytest.mark.parametrize("weights", [(1, 0, 0), (0, 1, 0), (0, 0, 1)])
def test_translation(small, weights):
    lat, R, params, G = small
    sel = [i for i, (n, c) in enumerate(params) if c < 3]
    pos = [params[i] for i in sel]
    g = G[sel, W3.index(weights)]
    tot = np.zeros(3)
    for (n, c), v in zip(pos, g):
        tot[c] += v
    expect = 2 * R.mesh.sum(axis=0) * weights[2]
    scale = np.abs(g).max()
    assert np.abs(tot - expect).max() <= 1e-6 * max(scale, np.abs(expect).max()), (tot, expect)
