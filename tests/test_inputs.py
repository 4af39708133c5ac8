"""The stored mock images equal what the oracle's synthesis writes from the seeds."""
import hashlib
import json
import os

import numpy as np
import pytest

import synthgen
from oracle import mock

DATA = os.path.join(os.path.dirname(__file__), "data")


@pytest.mark.parametrize("name", ["c1", "c2", "c4", "large"])
def test_stored_inputs(name):
    path = os.path.join(DATA, f"{name}.npz")
    with open(os.path.join(DATA, "MANIFEST.json")) as f:
        man = json.load(f)
    with open(path, "rb") as f:
        assert hashlib.sha256(f.read()).hexdigest() == man[f"{name}.npz"]
    z = np.load(path)
    D = mock.workload_data(synthgen.WORKLOADS[name])
    if name == "large":   # stored rounded to FP32
        assert z["d"].dtype == np.float32
        np.testing.assert_array_equal(z["d"], D["d"].astype(np.float32))
    else:
        np.testing.assert_allclose(z["d"], D["d"], rtol=0, atol=1e-12)
    assert float(z["sigma"]) == pytest.approx(D["sigma"], rel=1e-14)
    np.testing.assert_allclose(z["psf"], D["psf"], rtol=0, atol=1e-16)
