"""The device-side lattice generator reproduces latgen.bcc bit for bit."""

import numpy as np
import pytest

import latgen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("radius,jitter,seed", [
    (0.1, 0.0, 1),
    (("uniform", 0.05, 0.12), 0.05, 1),
    (("rel", 0.08, 0.1), 0.0, 3),
    (("rel", 0.08, 0.1), 0.01, 2),
])
def test_device_bcc_matches_host(radius, jitter, seed):
    import latgen.device

    host = latgen.bcc(5, radius=radius, jitter=jitter, seed=seed)
    dev = latgen.device.bcc(5, radius=radius, jitter=jitter, seed=seed)
    for f in ("x", "y", "z", "radius", "strut_a", "strut_b"):
        a = getattr(host, f)
        b = getattr(dev, f).cpu().numpy()
        assert a.dtype == b.dtype and np.array_equal(a.view(np.uint32) if a.dtype == np.float32 else a,
                                                     b.view(np.uint32) if b.dtype == np.float32 else b), f
