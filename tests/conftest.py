import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def c2_problem():
    import synthgen
    from oracle import mock, solve
    w = synthgen.C2
    D = mock.workload_data(w)
    pb = solve.Problem(D["lens"], D["d"], D["sigma"], D["psf"], w.nx, w.ny, w.pix,
                       w.nsub_model, w.ns, w.half_width, w.reg)
    return w, D, pb
