import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


class Box:
    """A plain attribute bag for hand-made fields and grids."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def make_lens(z, m, kappa_s, gamma):
    import numpy as np
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    m = np.broadcast_to(np.asarray(m, dtype=np.float64), z.shape).copy()
    return Box(x=z.real.copy(), y=z.imag.copy(), m=m, kappa_s=float(kappa_s),
               gamma=float(gamma))


@pytest.fixture
def lens_factory():
    return make_lens
