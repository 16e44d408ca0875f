"""The device-side lattice generator reproduces latgen.bcc bit for bit."""

import numpy as np
import pytest

import latgen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("radius,jitter,seed,order", [
    (0.1, 0.0, 1, "grid"),
    (("uniform", 0.05, 0.12), 0.05, 1, "grid"),
    (("rel", 0.08, 0.1), 0.0, 3, "grid"),
    (("rel", 0.08, 0.1), 0.01, 2, "grid"),
    (("rel", 0.08, 0.1), 0.0, 3, "layer"),
    (("uniform", 0.05, 0.12), 0.05, 1, "layer"),
])
def test_device_bcc_matches_host(radius, jitter, seed, order):
    import latgen.device

    host = latgen.bcc(5, radius=radius, jitter=jitter, seed=seed, order=order)
    dev = latgen.device.bcc(5, radius=radius, jitter=jitter, seed=seed, order=order)
    for f in ("x", "y", "z", "radius", "strut_a", "strut_b"):
        a = getattr(host, f)
        b = getattr(dev, f).cpu().numpy()
        assert a.dtype == b.dtype and np.array_equal(a.view(np.uint32) if a.dtype == np.float32 else a,
                                                     b.view(np.uint32) if b.dtype == np.float32 else b), f
